"""Pins of the oracle's ancestral sampler (the O(D) parallel generation that
Sec. 5 leaves to future work, run by the scheduler of Sec. 3).

A symbol is drawn as the inverse of its quantised CDF at a 16-bit slot: the
top 16 bits of word c of the Philox4x64-10 block (Salmon et al., SC'11) with
counter (y W + x, 0, 0, 0) and key (seed, 0). Pinned here by:
  * the generator against numpy's own Philox4x64-10 (independent code; numpy
    increments the counter before each block);
  * a model whose quantised CDF is known in closed form (all of F's mass in a
    tail bin), where every drawn symbol follows from the slot alone;
  * the inverse-CDF property against the oracle's CDF rows of the drawn
    image, slot by slot;
  * order independence: raster, wavefront and any later wavefront offset
    draw the same image (each pixel's slot depends on its position only);
  * a chi-square test of zero-context draws (1x1 patches) against the pmf
    freq / 2^16.
"""
import numpy as np
import pytest

import oracle
import synth
from sample_ref import U64, boundary_seeds, chi2_pvalue, closed_form_delta, decrement, numpy_slots


def model(name):
    b, _ = synth.model_blob(name)
    return oracle.Model.from_blob(b)


def test_philox_matches_numpy():
    keys = [(0, 0), (1, 0), (0xDEADBEEF12345678, 0), (2**64 - 1, 2**64 - 1)]
    ctrs = [(0, 0, 0, 0), (1, 0, 0, 0), (12345, 0, 0, 0), (0, 1, 0, 0), (2**64 - 1, 5, 7, 9), (3, 2**64 - 1, 0, 1)]
    for k in keys:
        for c in ctrs:
            g = np.random.Philox(key=np.array(k, dtype=U64), counter=decrement(c))
            assert np.array_equal(oracle.philox4x64(c, k), g.random_raw(4)), (k, c)


def test_slots_match_numpy():
    H, W, seed = 5, 7, 20220113
    ref = numpy_slots(seed, H, W)
    for y in range(H):
        for x in range(W):
            for c in range(3):
                assert oracle.sample_slot(seed, W, y, x, c) == ref[y, x, c]


@pytest.mark.parametrize("h", [1, 3])
def test_delta_model_closed_form(h):
    m = oracle.Model.from_params(h, 8, 0, synth.delta_params(h, 8))
    H, W, seed = 48, 40, 77
    want = closed_form_delta(numpy_slots(seed, H, W))
    # the tails are reached: some symbols other than the mode are drawn
    assert np.count_nonzero(want[..., 0]) > 0 and np.count_nonzero(want[..., 1] != 255) > 0
    for order in (0, 1):
        assert np.array_equal(m.sample(H, W, seed, order=order), want)
    assert np.array_equal(m.sample(H, W, seed, order=1, ph=16, pw=9), want)


def test_delta_model_boundaries():
    """Slots exactly on a bin boundary: cdf[v] <= slot < cdf[v + 1] decides."""
    m = oracle.Model.from_params(2, 8, 0, synth.delta_params(2, 8))
    for (ch, v), seed in boundary_seeds().items():
        slots = numpy_slots(seed, 8, 8)
        img = m.sample(8, 8, seed, order=1)
        assert np.array_equal(img, closed_form_delta(slots)), (ch, v, seed)


@pytest.mark.parametrize("name,ph,pw", [("tiny", 0, 0), ("tiny", 8, 5), ("C", 0, 0)])
def test_draws_are_inverse_cdf(name, ph, pw):
    m = model(name)
    H, W, seed = 12, 11, 5
    img = m.sample(H, W, seed, order=1, ph=ph, pw=pw)
    cdf = m.stats(img, ph=ph, pw=pw, cdf=True)["cdf"]  # rows given the drawn image
    slot = numpy_slots(seed, H, W)
    v = img.astype(np.int64)
    lo = np.take_along_axis(cdf, v[..., None], axis=3)[..., 0]
    hi = np.take_along_axis(cdf, v[..., None] + 1, axis=3)[..., 0]
    assert np.all(lo <= slot) and np.all(slot < hi)
    # a different seed draws a different image
    assert not np.array_equal(img, m.sample(H, W, seed + 1, order=1, ph=ph, pw=pw))


def test_order_independence():
    m = model("tiny")
    H, W, seed = 9, 13, 314
    ref = m.sample(H, W, seed, order=0)
    assert np.array_equal(m.sample(H, W, seed, order=1), ref)
    assert np.array_equal(m.sample(H, W, seed, offset=m.h + 2), ref)
    refp = m.sample(H, W, seed, order=0, ph=4, pw=6)
    assert np.array_equal(m.sample(H, W, seed, order=1, ph=4, pw=6), refp)


def test_non_causal_order_is_refused():
    """An offset below h + 1 would read a pixel not drawn yet: the oracle's
    poisoned canvas turns that into an error instead of a sample."""
    m = model("tiny")
    with pytest.raises(oracle.OracleError):
        m.sample(6, 9, 1, offset=m.h)


def test_zero_context_chi_square():
    """1x1 patches: every pixel is drawn at zero context, so R is i.i.d. with
    pmf freq / 2^16 of the zero-context row; G given R likewise."""
    m = model("tiny")
    H, W, seed = 64, 64, 99
    img = m.sample(H, W, seed, order=1, ph=1, pw=1)
    cdf = m.stats(np.zeros((1, 256, 3), dtype=np.uint8) + np.arange(256, dtype=np.uint8)[None, :, None],
                  ph=1, pw=1, cdf=True)["cdf"][0]  # row r: pixel (r, r, r) at zero context
    pmf_r = np.diff(cdf[0, 0]) / 65536.0
    p, nb = chi2_pvalue(np.bincount(img[..., 0].ravel(), minlength=256), pmf_r)
    assert nb > 10 and p > 1e-4, (p, nb)
    # G marginal: sum over r of p(r) p(g | r)
    pmf_g = sum(pmf_r[r] * np.diff(cdf[r, 1]) / 65536.0 for r in range(256))
    p, nb = chi2_pvalue(np.bincount(img[..., 1].ravel(), minlength=256), pmf_g)
    assert nb > 10 and p > 1e-4, (p, nb)
