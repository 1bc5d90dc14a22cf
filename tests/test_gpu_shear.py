"""GPU parity of the sheared-layout decoder (order 2: ShearLoC, Sec. 3.1,
Algorithm 2): the wavefront containers decoded with each pixel's context
gathered from a window of the lane's sheared canvas (step t = column t).

It must agree bit for bit with the unsheared wavefront decoder: the decoded
images equal the originals, the per-symbol (start, freq) it uses equal the
unsheared decoder's and the encoder's, for every model size, stream count and
lane shape (lanes narrower than h + 1, single rows and columns, lanes taller
than a wave, ragged patches), in the benchmark's full-size configuration, for
sampling, and under graph capture. The oracle's own sheared decoder is pinned
on the CPU (test_oracle_shear.py); here the FP64 oracle decodes the same
containers as a third opinion on small cases.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth

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


def cuda(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


def images(shapes, base):
    return [synth.smooth_field_image(2.0, 3, 2, H, W, base + k) for k, (H, W) in enumerate(shapes)]


CASES = [
    # model, shapes, patch, streams
    ("A", [(40, 70), (33, 17), (64, 64)], (32, 32), 1),
    ("A", [(40, 70), (33, 17)], (16, 24), 2),
    ("B", [(40, 70), (33, 17), (70, 50)], (32, 32), 4),
    ("B", [(70, 50), (9, 130)], None, 4),            # whole-image lanes, taller than a wave
    ("C", [(40, 70), (1, 29), (29, 1)], (16, 24), 4),  # h = 2, single rows and columns
    ("C", [(40, 70), (12, 11)], (7, 2), 1),          # lanes narrower than h + 1
    ("A", [(200, 9), (5, 300)], None, 2),            # tall and wide whole images
    ("B", [(40, 70), (33, 17), (86, 64)], (86, 64), 16),  # a stream per row of a group
    ("C", [(40, 70), (1, 29), (29, 1)], (16, 24), 8),    # rows p and p + 8 share a stream
]


@pytest.mark.parametrize("name,shapes,patch,K", CASES)
def test_sheared_decode_bitwise(nx, name, shapes, patch, K):
    say(f"[gpu] sheared decode: model {name}, {shapes}, patch {patch}, K {K}")
    m, _ = models(nx, name)
    imgs = images(shapes, 4000 + 7 * len(shapes))
    ts = [cuda(i) for i in imgs]
    data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=K)
    d2, o2 = m.encode(ts, order=nx.SHEARED, patch=patch, interleave=K)
    assert torch.equal(d2, data) and torch.equal(o2, offs)  # same containers
    out1, _, sym1 = m.decode(data, offs, shapes, order=nx.WAVEFRONT, patch=patch, interleave=K, trace=True)
    out2, _, sym2 = m.decode(data, offs, shapes, order=nx.SHEARED, patch=patch, interleave=K, trace=True)
    for a, b in zip(out2, ts):
        assert torch.equal(a, b)
    assert torch.equal(sym1, sym2)
    enc, _ = m.debug_symbols(ts, patch=patch)
    assert torch.equal(enc, sym2)


@pytest.mark.parametrize("patch", [None, (8, 6)])
def test_sheared_decode_vs_oracle_algorithm2(nx, patch):
    """The FP64 oracle's sheared decoder (Algorithm 2) on the oracle's own
    container of the same image, next to the GPU's sheared decode."""
    say(f"[gpu] sheared decode vs oracle Algorithm 2, patch {patch}")
    m, om = models(nx, "C")
    img = images([(14, 19)], 4500)[0]
    ph, pw = (0, 0) if patch is None else patch
    o_dec = om.decode_shear(om.encode(img, order=1, ph=ph, pw=pw), 14, 19, ph, pw)
    data, offs = m.encode([cuda(img)], order=nx.SHEARED, patch=patch)
    (g_dec,), _ = m.decode(data, offs, [(14, 19)], order=nx.SHEARED, patch=patch)
    assert np.array_equal(o_dec, img)
    assert np.array_equal(g_dec.cpu().numpy(), img)


def test_sheared_full_size(nx):
    """The benchmark configuration: 4 x 1024^2 + 2 x 2048x1536, model B, the
    benchmark's patches (tune.balanced_patch), four streams, decoded in the
    sheared layout."""
    from paper_2201_05213_amd import tune

    say("[gpu] sheared decode: full-size batch")
    m, _ = models(nx, "B")
    ts = [cuda(i) for i in synth.workload_images("large6")]
    shapes = [tuple(t.shape[:2]) for t in ts]
    patch = tune.balanced_patch(shapes)
    data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=4)
    out, st = m.decode(data, offs, shapes, order=nx.SHEARED, patch=patch, interleave=4)
    assert int(st.abs().sum()) == 0
    for a, b in zip(out, ts):
        assert torch.equal(a, b)


def test_sheared_sampling(nx):
    say("[gpu] sheared sampling equals unsheared sampling")
    m, _ = models(nx, "A")
    shapes, seeds = [(37, 45), (64, 64), (3, 70)], [5, 6, 7]
    for patch in (None, (16, 16)):
        a = m.sample(shapes, seeds, order=nx.WAVEFRONT, patch=patch)
        b = m.sample(shapes, seeds, order=nx.SHEARED, patch=patch)
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def test_sheared_graph_replay(nx):
    """prepare/run with order 2 captured in a graph: every replay decodes the
    containers copied into the captured buffers (the kernel clears its own
    windows, so no memset is recorded)."""
    say("[gpu] sheared decode: graph capture and replays")
    m, _ = models(nx, "A")
    shapes = [(48, 40), (33, 17)]
    sets = [images(shapes, 4600 + 10 * r) for r in range(3)]
    enc = [m.encode([cuda(i) for i in s], order=nx.SHEARED, patch=(16, 16), interleave=2) for s in sets]
    cap = max(int(d.numel()) for d, _ in enc)
    data = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    offs = torch.zeros(len(shapes) + 1, dtype=torch.int64, device="cuda")
    out = [torch.empty((H, W, 3), dtype=torch.uint8, device="cuda") for H, W in shapes]
    status = torch.empty(len(shapes), dtype=torch.int32, device="cuda")
    plan, ws = m.decode_prepare(out, order=nx.SHEARED, patch=(16, 16), interleave=2)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.decode_run(plan, data, offs, status, ws)
    torch.cuda.synchronize()
    for r in (0, 1, 2, 1):
        d, o = enc[r]
        data[:d.numel()].copy_(d)
        offs.copy_(o)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(status.abs().sum()) == 0
        for a, b in zip(out, sets[r]):
            assert np.array_equal(a.cpu().numpy(), b), r


def test_order_out_of_range_is_refused(nx):
    from paper_2201_05213_amd import NelloxError

    m, _ = models(nx, "A")
    t = cuda(images([(8, 8)], 4700)[0])
    with pytest.raises(NelloxError):
        m.encode([t], order=3)
