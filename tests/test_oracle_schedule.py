"""Pins of the decode schedule (Sec. 3, Fig. 3) and of the oracle's orders.

The step of a pixel is derived here by brute force from the dependency set
of Eq. (3) alone (longest path in the dependency DAG), then compared with the
paper's printed table, its closed forms and the oracle's decode order.
"""
import numpy as np
import pytest

import oracle


def deps(i, j, h, H, W):
    """Dependencies of pixel (i, j) under Eq. (3): rows i-h..i-1, columns
    j-h..j+h, plus row i, columns j-h..j-1, restricted to the image."""
    out = []
    for y in range(i - h, i):
        for x in range(j - h, j + h + 1):
            if 0 <= y < H and 0 <= x < W:
                out.append((y, x))
    for x in range(j - h, j):
        if 0 <= x < W:
            out.append((i, x))
    return out


def earliest_steps(H, W, h):
    """Earliest parallel step of every pixel (0-based): 0 without
    dependencies, else 1 + the latest dependency. Raster order is a
    topological order of the DAG, so one pass suffices."""
    s = np.zeros((H, W), dtype=np.int64)
    for i in range(H):
        for j in range(W):
            d = deps(i, j, h, H, W)
            s[i, j] = 1 + max(s[y, x] for y, x in d) if d else 0
    return s


def test_fig3_table(golden):
    table = np.array([[int(v) for v in row] for row in golden("fig3_topological_order_5x5_h1.txt")])
    s = earliest_steps(5, 5, 1)
    assert (s + 1 == table).all()
    # text of Sec. 3: 13 steps instead of 25, pixels (2,4) and (3,2) (1-indexed) both at step 6
    assert s.max() + 1 == 13 == oracle.steps(5, 5, 1)
    assert table[1, 3] == table[2, 1] == 6


@pytest.mark.parametrize("H,W,h", [(5, 5, 1), (32, 32, 3), (9, 13, 2), (13, 9, 2), (1, 7, 3), (7, 1, 3),
                                   (64, 64, 3), (8, 40, 3), (64, 32, 3), (20, 20, 1)])
def test_closed_forms_vs_brute_force(H, W, h):
    s = earliest_steps(H, W, h)
    # step formula t = j + (h+1) i (Sec. 3, with 0-based indices)
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    t = jj + (h + 1) * ii
    # it is a valid schedule for every shape: each dependency comes earlier
    for i in range(H):
        for j in range(W):
            assert all(t[y, x] < t[i, j] for y, x in deps(i, j, h, H, W))
    if W >= h + 1:
        # and the earliest one once a row is at least h+1 wide; narrower
        # lanes (ragged patch edges) could go faster, the formula is kept
        assert (s == t).all()
    else:
        assert (s <= t).all()
    T = int(t.max()) + 1
    assert T == W + (h + 1) * (H - 1) == oracle.steps(H, W, h)
    width = np.bincount(t.ravel()).max()
    assert width == min(H, (W + h) // (h + 1))
    assert np.bincount(t.ravel()).sum() == H * W


def test_square_closed_forms_paper():
    # Sec. 3: T = D + (D-1)(h+1) on floor((D+h)/(h+1)) units
    for D in (5, 32, 64, 128, 1024):
        for h in (1, 2, 3):
            assert oracle.steps(D, D, h) == D + (D - 1) * (h + 1)


@pytest.mark.parametrize("H,W,h", [(5, 5, 1), (8, 11, 3), (11, 8, 2), (1, 1, 3)])
def test_oracle_orders(H, W, h):
    # raster order: every (pixel, channel) once in row-major order
    r = oracle.symbol_order(H, W, 0)
    assert len(r) == 3 * H * W
    assert [tuple(x) for x in r] == [(i, j, c) for i in range(H) for j in range(W) for c in range(3)]
    # wavefront order with offset h+1 is a topological order of the DAG
    w = oracle.symbol_order(H, W, h + 1)
    assert len(w) == 3 * H * W and len({tuple(x) for x in w}) == 3 * H * W
    pos = {}
    for n, (i, j, c) in enumerate(w):
        pos[(i, j, c)] = n
    for i in range(H):
        for j in range(W):
            for y, x in deps(i, j, h, H, W):
                assert pos[(y, x, 2)] < pos[(i, j, 0)]
            assert pos[(i, j, 0)] < pos[(i, j, 1)] < pos[(i, j, 2)]
    # steps are non-decreasing along the sequence and equal j + (h+1) i
    t = w[:, 1] + (h + 1) * w[:, 0]
    assert (np.diff(t) >= 0).all()


def test_offset_h_is_not_causal():
    # with step j + h i, pixel (i-1, j+h) shares the step of (i, j)
    h, H, W = 2, 6, 7
    w = oracle.symbol_order(H, W, h)
    pos = {tuple(x): n for n, x in enumerate(w)}
    violated = any(pos[(y, x, 2)] > pos[(i, j, 0)]
                   for i in range(H) for j in range(W) for y, x in deps(i, j, h, H, W))
    assert violated
