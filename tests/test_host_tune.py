"""Host logic of the patch chooser: lane counts and the balanced patch
height (no GPU; the CU count is given)."""
import itertools
import math

import pytest

import synth
from paper_2201_05213_amd import tune


def test_lane_count_brute_force():
    shapes = [(37, 29), (64, 64), (1, 200), (130, 7)]
    for patch in itertools.product((1, 5, 16, 64, 100), (3, 16, 64)):
        ph, pw = patch
        n = 0
        for H, W in shapes:  # count the tiles one by one
            for y in range(0, H, ph):
                for x in range(0, W, pw):
                    n += 1
        assert tune.lane_count(shapes, patch) == n


@pytest.mark.parametrize("cus", [256, 304, 80])
def test_balanced_patch_is_the_shortest_that_fits(cus):
    shapes = synth.workload_shapes("large6")
    ph, pw = tune.balanced_patch(shapes, cus=cus)
    cap = 2 * 4 * cus
    assert pw == 64
    assert tune.lane_count(shapes, (ph, pw)) <= cap or ph == 2048
    for H, _ in shapes:
        if H > ph:
            assert H - (math.ceil(H / ph) - 1) * ph >= ph / 2
    # every shorter height (from the floor of 64 rows) breaks a rule
    for short in range(64, ph):
        tails_ok = all(H <= short or H - (math.ceil(H / short) - 1) * short >= short / 2 for H, _ in shapes)
        assert tune.lane_count(shapes, (short, 64)) > cap or not tails_ok


def test_balanced_patch_large_batch_on_256_cus():
    # 4 x 1024^2 + 2 x 2048x1536 on 256 CUs: 84 and 85 rows fit 2,048 lanes
    # but leave 16- and 4-row ragged lanes; 86 rows give 1,920 full lanes
    shapes = synth.workload_shapes("large6")
    assert tune.balanced_patch(shapes, cus=256) == (86, 64)
    assert tune.lane_count(shapes, (86, 64)) == 1920
    assert tune.lane_count(shapes, (84, 64)) == 2032
    # a batch far below the cap takes the floor
    assert tune.balanced_patch([(1024, 1024)], cus=256) == (64, 64)
