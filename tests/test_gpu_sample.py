"""GPU parity of the ancestral sampler (nellox_sample through the C ABI): the
O(D) parallel generation that Sec. 5 leaves to future work, run by the
wavefront schedule of Sec. 3.

Checks, against references that share no code with the HIP path:
  * the tail-mass model, whose draws follow from the slots in closed form
    (numpy's Philox), including slots exactly on bin boundaries;
  * every drawn symbol is the inverse of the GPU's own quantised CDF (the
    encoder's rows of the drawn image) at the numpy Philox slot;
  * the oracle's teacher-forced choice at every symbol, and the oracle's own
    sample, equal the GPU's (a difference is allowed only where the slot sits
    on a CDF boundary that the FP32 and FP64 rows place one count apart);
  * order, batch and launch independence; a chi-square test of zero-context
    draws; the full-size batch of the benchmark, checked symbol by symbol
    and on oracle-computed patches, then coded and decoded back exactly.
"""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from sample_ref import boundary_seeds, chi2_pvalue, closed_form_delta, numpy_slots

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def nx():
    import paper_2201_05213_amd as nx

    torch.cuda.set_device(0)
    return nx


_MODELS = {}


def models(nx, name):
    if name not in _MODELS:
        blob, _ = synth.model_blob(name)
        _MODELS[name] = (nx.Model(blob), oracle.Model.from_blob(blob))
    return _MODELS[name]


def delta_model(nx, h):
    blob = synth.write_blob(h, 8, 0, synth.delta_params(h, 8))
    return nx.Model(blob)


def host(t):
    return t.cpu().numpy()


def symbols_of(m, imgs, patch):
    """(start, freq) arrays per image from the encoder's pass over `imgs`."""
    sym, _ = m.debug_symbols(imgs, patch=patch)
    s = host(sym).view(np.uint32)
    out, o = [], 0
    for t in imgs:
        H, W = int(t.shape[0]), int(t.shape[1])
        blk = s[o:o + H * W * 3].reshape(H, W, 3)
        out.append(((blk & 0xFFFF).astype(np.int64), (blk >> 16).astype(np.int64)))
        o += H * W * 3
    return out


def check_inverse_cdf(m, imgs, seeds, patch):
    """Every drawn symbol v satisfies start_v <= slot < start_v + freq_v with
    the GPU's own rows (the encoder's, bitwise equal to the decoder's)."""
    for t, (start, freq), seed in zip(imgs, symbols_of(m, imgs, patch), seeds):
        slot = numpy_slots(seed, int(t.shape[0]), int(t.shape[1]))
        # freq 0 stands for 2^16 (a row with all mass in one bin cannot occur: freq <= 65281)
        assert np.all(freq >= 1)
        assert np.all(start <= slot) and np.all(slot < start + freq)


def oracle_choice(om, img, seed, ph, pw, W_full=None, y0=0, x0=0):
    """The oracle's inverse CDF at each slot, its rows conditioned on the
    drawn image (teacher forcing), and the rows themselves."""
    cdf = om.stats(img, ph=ph, pw=pw, cdf=True)["cdf"].astype(np.int64)
    H, W = img.shape[:2]
    if W_full is None:
        slot = numpy_slots(seed, H, W)
    else:
        slot = numpy_slots(seed, y0 + H, W_full)[y0:y0 + H, x0:x0 + W]
    v = (cdf[..., 1:] <= slot[..., None]).sum(-1)
    return v, cdf, slot


def explained(got, v, cdf, slot):
    """Positions where the oracle's choice differs from the GPU's; each one
    must sit on a boundary of the GPU's bin in the oracle's row (within one
    count), where FP32 and FP64 quantisation may disagree by one."""
    bad = np.argwhere(got.astype(np.int64) != v)
    for (y, x, c) in bad:
        g = int(got[y, x, c])
        s = int(slot[y, x, c])
        lo, hi = int(cdf[y, x, c, g]), int(cdf[y, x, c, g + 1])
        assert abs(s - lo) <= 1 or abs(s - hi) <= 1, (y, x, c, g, s, lo, hi)
    return len(bad)


@pytest.mark.parametrize("h", [1, 2, 3])
def test_delta_model_closed_form(nx, h):
    say(f"[gpu] sample: tail-mass model h={h}, closed form")
    m = delta_model(nx, h)
    shapes = [(64, 64), (1, 1), (1, 37), (29, 1), (8, 8)]
    seeds = [77, 5, 6, 7, 8]
    for order, patch in [(1, None), (0, None), (1, (16, 9)), (1, (1, 1))]:
        out = m.sample(shapes, seeds, order=order, patch=patch)
        torch.cuda.synchronize()
        for t, (H, W), sd in zip(out, shapes, seeds):
            assert np.array_equal(host(t), closed_form_delta(numpy_slots(sd, H, W))), (order, patch, H, W)


def test_delta_model_boundaries(nx):
    say("[gpu] sample: slots on bin boundaries")
    m = delta_model(nx, 2)
    bs = boundary_seeds()
    seeds = list(bs.values())
    out = m.sample([(8, 8)] * len(seeds), seeds)
    for t, sd in zip(out, seeds):
        assert np.array_equal(host(t), closed_form_delta(numpy_slots(sd, 8, 8))), sd


@pytest.mark.parametrize("name", ["A", "B", "C"])
@pytest.mark.parametrize("order,patch", [(1, None), (1, (16, 24)), (0, (8, 8))])
def test_draws_are_inverse_of_gpu_cdf(nx, name, order, patch):
    say(f"[gpu] sample: inverse CDF, model {name}, order {order}, patch {patch}")
    m, _ = models(nx, name)
    shapes, seeds = [(40, 52), (17, 33), (1, 5)], [11, 12, 13]
    out = m.sample(shapes, seeds, order=order, patch=patch)
    check_inverse_cdf(m, out, seeds, patch)


@pytest.mark.parametrize("name", ["A", "B", "C"])
@pytest.mark.parametrize("patch", [None, (8, 8)])
def test_matches_oracle(nx, name, patch):
    say(f"[gpu] sample vs oracle, model {name}, patch {patch}")
    m, om = models(nx, name)
    shapes, seeds = [(24, 20), (9, 31)], [2022, 5]
    ph, pw = (0, 0) if patch is None else patch
    out = m.sample(shapes, seeds, patch=patch)
    n_syms = n_bad = 0
    for t, (H, W), sd in zip(out, shapes, seeds):
        got = host(t)
        v, cdf, slot = oracle_choice(om, got, sd, ph, pw)
        nb = explained(got, v, cdf, slot)
        n_syms += got.size
        n_bad += nb
        if nb == 0:
            # the same conditionals at every symbol: the oracle's own sample is identical
            assert np.array_equal(om.sample(H, W, sd, order=1, ph=ph, pw=pw), got)
    say(f"  symbols {n_syms}, on a one-count boundary {n_bad}")
    assert n_bad <= max(1, n_syms // 10000)


def test_order_batch_and_launch_independence(nx):
    say("[gpu] sample: order / batch independence")
    m, _ = models(nx, "A")
    shapes, seeds = [(37, 45), (20, 30), (37, 45)], [1, 2, 1]
    for patch in (None, (16, 16)):
        a = m.sample(shapes, seeds, order=1, patch=patch)
        b = m.sample(shapes, seeds, order=0, patch=patch)
        for x, y in zip(a, b):
            assert torch.equal(x, y)
        assert torch.equal(a[0], a[2])
        (one,) = m.sample([shapes[1]], [seeds[1]], patch=patch)
        assert torch.equal(one, a[1])
        (other,) = m.sample([shapes[1]], [3], patch=patch)
        assert not torch.equal(other, a[1])


def test_zero_context_chi_square(nx):
    """1x1 patches: 65536 pixels drawn at zero context; R and G marginals
    against the oracle's pmf freq / 2^16."""
    say("[gpu] sample: chi-square at zero context, 256x256, 1x1 patches")
    m, om = models(nx, "A")
    (t,) = m.sample([(256, 256)], [2024], patch=(1, 1))
    img = host(t)
    probe = np.zeros((1, 256, 3), dtype=np.uint8) + np.arange(256, dtype=np.uint8)[None, :, None]
    cdf = om.stats(probe, ph=1, pw=1, cdf=True)["cdf"][0].astype(np.int64)
    pmf_r = np.diff(cdf[0, 0]) / 65536.0
    p_r, nb_r = chi2_pvalue(np.bincount(img[..., 0].ravel(), minlength=256), pmf_r)
    pmf_g = sum(pmf_r[r] * np.diff(cdf[r, 1]) / 65536.0 for r in range(256))
    p_g, nb_g = chi2_pvalue(np.bincount(img[..., 1].ravel(), minlength=256), pmf_g)
    say(f"  R: p = {p_r:.3f} over {nb_r} bins; G: p = {p_g:.3f} over {nb_g} bins")
    assert nb_r > 10 and p_r > 1e-4
    assert nb_g > 10 and p_g > 1e-4


def test_edges_and_errors(nx):
    say("[gpu] sample: empty batch, argument errors")
    from paper_2201_05213_amd import _lib

    m, _ = models(nx, "A")
    assert m.sample([], []) == []
    L = _lib.load()
    img = torch.empty((8, 8, 3), dtype=torch.uint8, device="cuda")
    arr = (_lib.NelloxImage * 1)(_lib.NelloxImage(img.data_ptr(), 8, 8))
    o = _lib.NelloxOpts(1, 0, 0, 1)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    seeds = (ctypes.c_uint64 * 1)(1)
    st = lambda *a: L.nellox_sample(m._h, *a)  # noqa: E731
    assert st(1, None, ctypes.byref(o), arr, ws.data_ptr(), ws.numel(), None) == 1  # null seeds
    assert st(1, seeds, None, arr, ws.data_ptr(), ws.numel(), None) == 1  # null opts
    bad = _lib.NelloxOpts(3, 0, 0, 1)
    assert st(1, seeds, ctypes.byref(bad), arr, ws.data_ptr(), ws.numel(), None) == 1  # bad order
    assert st(1, seeds, ctypes.byref(o), arr, ws.data_ptr(), 16, None) == 3  # workspace too small
    assert st(1, seeds, ctypes.byref(o), arr, None, ws.numel(), None) == 1  # null workspace
    assert st(1, seeds, ctypes.byref(o), arr, ws.data_ptr(), ws.numel(), None) == 0
    torch.cuda.synchronize()


def test_full_size_batch(nx):
    """The benchmark's batch shape (4 x 1024^2 + 2 x 2048x1536, model B,
    the benchmark's patches, wavefront): every symbol against the GPU's own
    CDF, a few patches against the oracle, and the sample coded and decoded
    back."""
    from paper_2201_05213_amd import tune

    m, om = models(nx, "B")
    shapes = synth.workload_shapes("large6")
    seeds = [900 + k for k in range(len(shapes))]
    ph, pw = tune.balanced_patch(shapes)
    say(f"[gpu] sample: full-size batch, model B, patch {ph}x{pw}")
    out = m.sample(shapes, seeds, patch=(ph, pw))
    torch.cuda.synchronize()
    check_inverse_cdf(m, out, seeds, (ph, pw))
    say("  inverse-CDF property holds on every symbol")
    rng = np.random.Generator(np.random.PCG64(4))
    n_bad = n_syms = 0
    for k in (0, 5):
        H, W = shapes[k]
        full = host(out[k])
        for _ in range(2):
            py = int(rng.integers(0, -(-H // ph))) * ph
            px = int(rng.integers(0, -(-W // pw))) * pw
            crop = np.ascontiguousarray(full[py:py + ph, px:px + pw])
            v, cdf, slot = oracle_choice(om, crop, seeds[k], 0, 0, W_full=W, y0=py, x0=px)
            n_bad += explained(crop, v, cdf, slot)
            n_syms += crop.size
    say(f"  oracle patches: {n_syms} symbols, {n_bad} on a one-count boundary")
    assert n_bad <= max(1, n_syms // 10000)
    data, offs = m.encode(out, patch=(ph, pw), interleave=4)
    back, _ = m.decode(data, offs, shapes, patch=(ph, pw), interleave=4)
    for a, b in zip(out, back):
        assert torch.equal(a, b)
