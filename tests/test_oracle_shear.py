"""Pins of the oracle's sheared model (Sec. 3.1, ShearLoC, Algorithm 2).

  * the shear of a 5x5 label image with h = 1 is the matrix of Fig. 4b;
  * the sheared kernels of h = 1 and h = 2 are those of Fig. 5b / 5d;
  * the sheared length L = W + (h+1)(H-1) equals the step count T of the
    wavefront schedule, and column t of the sheared image holds exactly the
    pixels of step t (brute-force earliest steps from Eq. 3's dependencies);
  * the sheared kernel, mapped back to image offsets, is exactly the causal
    neighbourhood of Eq. 3, and reads only columns before the pixel's own;
  * unshear(shear(x)) = x;
  * the logits of every pixel computed in the sheared model are bitwise those
    of the unsheared model;
  * decoding a wavefront container column by column on the sheared canvas
    (NaN-poisoned where not decoded) returns the image.
"""
import numpy as np
import pytest

import oracle
import synth
from test_oracle_schedule import deps, earliest_steps


def label_image(H, W):
    return np.array([[10 * (i + 1) + (j + 1) for j in range(W)] for i in range(H)], dtype=np.float64)


def read_blocks(rows):
    """Golden rows split at 'h=<n>' markers -> {h: int matrix}."""
    out, cur, h = {}, [], None
    for r in rows:
        if r[0].startswith("h="):
            if h is not None:
                out[h] = np.array(cur, dtype=np.int64)
            h, cur = int(r[0][2:]), []
        else:
            cur.append([int(v) for v in r])
    out[h] = np.array(cur, dtype=np.int64)
    return out


def test_fig4b_sheared_image(golden):
    want = np.array([[int(v) for v in row] for row in golden("fig4b_sheared_5x5_h1.txt")])
    got = oracle.shear(label_image(5, 5), 2)
    assert got.shape == (5, 13)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("h", [1, 2])
def test_fig5bd_sheared_kernels(golden, h):
    want = read_blocks(golden("fig5bd_sheared_kernels.txt"))[h]
    K = 2 * h + 1
    # a one-channel model whose first kernel holds the labels w_ab of the live
    # taps (row a, b-th live column of that row, 1-indexed)
    C = 1
    conv = np.zeros((C, 3, K, K))
    for a in range(h + 1):
        b = 0
        for dx in range(K):
            if oracle.tap_live(h, a, dx):
                b += 1
                conv[0, 0, a, dx] = 10 * (a + 1) + b
    params = np.zeros(int(synth.param_count(h, C, 0)))
    params[:conv.size] = conv.ravel()
    m = oracle.Model.from_params(h, C, 0, params)
    Kp = m.shear_kernel()[0, 0]
    assert Kp.shape == (h + 1, h * (h + 2))
    assert np.array_equal(Kp.astype(np.int64), want)
    # the support function agrees with the kernel
    sup = np.array([[oracle.shear_tap_live(h, a, q) for q in range(h * (h + 2))] for a in range(h + 1)])
    assert np.array_equal(sup, want != 0)


@pytest.mark.parametrize("h", [1, 2, 3])
@pytest.mark.parametrize("H,W", [(1, 1), (5, 5), (4, 9), (9, 4), (7, 2), (3, 11)])
def test_columns_are_wavefront_steps(h, H, W):
    o = h + 1
    L = W + o * (H - 1)
    assert L == oracle.steps(H, W, h)  # L = T
    S = oracle.shear(np.arange(1, H * W + 1, dtype=np.float64).reshape(H, W), o)
    assert S.shape == (H, L)
    # the wavefront step j + o i; for lanes at least h + 1 wide it is the
    # earliest step of the dependency DAG
    steps = np.array([[j + o * i for j in range(W)] for i in range(H)])
    if W >= h + 1:
        assert np.array_equal(steps, earliest_steps(H, W, h))
    for t in range(L):
        col = {int(v) for v in S[:, t] if v != 0}
        want = {i * W + j + 1 for i in range(H) for j in range(W) if steps[i, j] == t}
        assert col == want, t
    assert np.array_equal(oracle.unshear(S, W, o), np.arange(1, H * W + 1).reshape(H, W))


@pytest.mark.parametrize("h", [1, 2, 3])
def test_sheared_kernel_is_the_causal_neighbourhood(h):
    """Map each live tap (a, q) of the sheared kernel back to an image offset
    of the pixel at sheared column t: row i - h + a, column
    (t - Q + q) - o (i - h + a) - j. The set must be Eq. 3's dependency set,
    and every tap must read an earlier column."""
    o, Q = h + 1, h * (h + 2)
    taps = set()
    for a in range(h + 1):
        for q in range(Q):
            if oracle.shear_tap_live(h, a, q):
                assert q - Q < 0
                dy = a - h
                dx = (q - Q) - o * dy
                taps.add((dy, dx))
    H = W = 4 * h + 3
    i, j = 2 * h + 1, 2 * h + 1
    want = {(y - i, x - j) for y, x in deps(i, j, h, H, W)}
    assert taps == want


@pytest.mark.parametrize("name", ["tiny", "C"])
def test_sheared_logits_bitwise(name):
    b, _ = synth.model_blob(name)
    m = oracle.Model.from_blob(b)
    for k, (H, W) in enumerate([(9, 13), (5, 3), (1, 7), (6, 1)]):
        img = synth.smooth_field_image(2.0, 3, 2, H, W, 700 + k)
        assert np.array_equal(m.theta_image_shear(img), m.theta_image(img)), (H, W)


@pytest.mark.parametrize("ph,pw", [(0, 0), (6, 5), (3, 9)])
def test_algorithm2_decode(ph, pw):
    b, _ = synth.model_blob("tiny")
    m = oracle.Model.from_blob(b)
    for k, (H, W) in enumerate([(12, 10), (7, 3), (1, 9), (9, 1)]):
        img = synth.smooth_field_image(2.0, 3, 2, H, W, 800 + k)
        data = m.encode(img, order=1, ph=ph, pw=pw)
        # the container's lane table follows the oracle's own format
        assert np.array_equal(m.decode_shear(data, H, W, ph, pw), img)


def test_algorithm2_rejects_corrupt_stream():
    b, _ = synth.model_blob("tiny")
    m = oracle.Model.from_blob(b)
    img = synth.smooth_field_image(2.0, 3, 2, 8, 8, 900)
    data = bytearray(m.encode(img, order=1))
    data[-3] ^= 0x5A
    with pytest.raises(oracle.OracleError):
        m.decode_shear(bytes(data), 8, 8)
