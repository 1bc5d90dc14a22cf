"""Host logic of the patch chooser: lane counts and the balanced patch
height (no GPU; the CU count is given)."""
import itertools
import math

import pytest

import synth
from paper_2201_05213_amd import ROWS, tune


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
            assert H - (math.ceil(H / ph) - 1) * ph >= ph / 4
    # every shorter height (from the floor of 64 rows) breaks a rule
    for short in range(64, ph):
        tails_ok = all(H <= short or H - (math.ceil(H / short) - 1) * short >= short / 4 for H, _ in shapes)
        assert tune.lane_count(shapes, (short, 64)) > cap or not tails_ok


def test_balanced_patch_large_batch_on_256_cus():
    # 4 x 1024^2 + 2 x 2048x1536 on 256 CUs: 80 and 81 rows need 2,080
    # lanes; 82 rows fit 2,032 (ragged lane rows of 40 and 80); with the old
    # half-lane tail rule 84 and 85 (16- and 4-row tails) and 82, 83 were
    # skipped for 86 rows, 1,920 lanes on 240 CUs
    shapes = synth.workload_shapes("large6")
    assert tune.balanced_patch(shapes, cus=256) == (82, 64)
    assert tune.lane_count(shapes, (81, 64)) == 2080
    assert tune.lane_count(shapes, (82, 64)) == 2032
    assert tune.lane_count(shapes, (86, 64)) == 1920
    assert tune.balanced_patch(shapes, cus=256, min_tail=0.5) == (86, 64)
    # a batch far below the cap takes the floor
    assert tune.balanced_patch([(1024, 1024)], cus=256) == (64, 64)


@pytest.mark.parametrize("K,bpd", [(16, 9.0), (16, 4.35), (8, 4.35), (4, 1.0)])
def test_balanced_patch_stream_budget(K, bpd):
    """With an expected bits/dim, a height is taken only if a full lane's K
    streams cost at most 0.1% of its bits; every shorter height from 64 rows
    breaks one of the rules."""
    shapes = synth.workload_shapes("large6")
    ph, pw = tune.balanced_patch(shapes, cus=256, interleave=K, bits_per_dim=bpd)
    cap = 2 * 4 * 256

    def fine(r):
        tails = all(H <= r or H - (math.ceil(H / r) - 1) * r >= r / 4 for H, _ in shapes)
        budget = K * tune.STREAM_BITS <= 1e-3 * 3 * r * 64 * bpd
        return tune.lane_count(shapes, (r, 64)) <= cap and tails and budget

    assert fine(ph)
    assert not any(fine(r) for r in range(64, ph))
    if (K, bpd) == (16, 9.0):
        assert ph == 82  # the random-init model's ~9 bits/dim leaves the benchmark's patch
    if (K, bpd) == (16, 4.35):
        assert ph >= 96  # 80 bits per lane need at least 95.8 rows of 64 columns at 4.35 bits/dim


def test_image_streams_count():
    for (H, W), patch in itertools.product([(37, 29), (64, 64), (1, 200), (130, 7)],
                                           [None, (1, 1), (16, 16), (64, 8)]):
        lanes = tune.lane_count([(H, W)], (H, W) if patch is None else patch)
        for K in (1, 2, 4, 8, 16):
            assert tune.image_streams(H, W, patch, K) == lanes * K
        # row streams: one per row of every lane
        ph, pw = (H, W) if patch is None else patch
        rows = sum(min(ph, H - y) for y in range(0, H, ph) for _ in range(0, W, pw))
        assert tune.image_streams(H, W, patch, ROWS) == rows
