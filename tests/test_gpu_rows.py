"""Row streams (interleave = -1): one rANS stream per lane row, decoded in
bands of 16 rows (a workgroup of four waves per band: the network split by
output tiles, 16 lanes per pixel for the mixture and the pops), every row of
a wavefront step at once (Sec. 3, Algorithm 1 with the whole step in
parallel), bands pipelined across workgroups.

Against the encoder (the decoder's (start, freq) bitwise the encoder's) and
the FP64 oracle (coded bits within 0.1% of its quantised ideal on whole
images): exact round trips for lanes shorter than a band, one row past a
band, many bands, lanes narrower than h + 1 columns, patches, mixed batches;
damaged containers reported, never a wrong image with status 0; prepared
(capturable) runs and the no-allocation entry point.
"""
import ctypes
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


@pytest.fixture(scope="module")
def models(nx):
    out = {}
    for name in ("A", "B", "C"):
        blob, _ = synth.model_blob(name)
        out[name] = (nx.Model(blob), blob)
    return out


def cuda(img):
    return torch.from_numpy(np.ascontiguousarray(img)).cuda()


SHAPES = [(1, 1), (1, 9), (9, 1), (5, 3), (16, 33), (17, 40), (32, 7), (64, 50), (65, 50), (130, 70), (200, 3),
          (3, 200)]


@pytest.mark.parametrize("name", ["A", "C"])
@pytest.mark.parametrize("shape", SHAPES)
def test_round_trip_and_symbols(models, nx, name, shape):
    say(f"[gpu] row streams, model {name}, {shape}")
    m, _ = models[name]
    H, W = shape
    img = synth.smooth_field_image(2.0, 3, 2, H, W, 8000 + H * 7 + W)
    t = cuda(img)
    data, offs = m.encode([t], order=nx.WAVEFRONT, interleave=nx.ROWS)
    assert nx.peek(data.cpu().numpy().tobytes())[4] == -1
    out, st, dump = m.decode(data, offs, [(H, W)], order=nx.WAVEFRONT, interleave=nx.ROWS, trace=True)
    assert int(st[0]) == 0 and torch.equal(out[0], t)
    sym, _ = m.debug_symbols([t])
    assert torch.equal(sym, dump)


@pytest.mark.parametrize("patch", [None, (100, 260), (64, 64), (70, 33)])
def test_batch_and_patches(models, nx, patch):
    """A batch of images of several sizes in one call, whole-image lanes and
    patch grids (lanes of several bands, ragged patch rows and columns)."""
    say(f"[gpu] row streams, batch, patch {patch}")
    m, _ = models["B"]
    shapes = [(300, 260), (64, 64), (129, 17), (1, 40), (40, 1)]
    imgs = [synth.smooth_field_image(2.0, 3, 2, H, W, 8100 + k) for k, (H, W) in enumerate(shapes)]
    ts = [cuda(i) for i in imgs]
    data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=nx.ROWS)
    out, st, dump = m.decode(data, offs, shapes, order=nx.WAVEFRONT, patch=patch, interleave=nx.ROWS, trace=True)
    assert int(st.abs().sum()) == 0
    for a, b in zip(out, ts):
        assert torch.equal(a, b)
    sym, _ = m.debug_symbols(ts, patch=patch)
    assert torch.equal(sym, dump)


def test_bits_against_oracle(models, nx):
    """Whole-image lanes, one stream per row: coded bits within 0.1% of the
    oracle's quantised ideal (a stream costs ~5 bits; a 256-pixel row carries
    about 6.9 kbit at 9 bits/dim)."""
    m, blob = models["B"]
    om = oracle.Model.from_blob(blob)
    imgs = [synth.smooth_field_image(4.0, 20, 3, 96, 256, 8200), synth.smooth_field_image(2.0, 3, 0, 128, 200, 8201)]
    ts = [cuda(i) for i in imgs]
    data, offs = m.encode(ts, order=nx.WAVEFRONT, interleave=nx.ROWS)
    got = float(sum(nx.payload_bits(data, offs)))
    ideal = sum(om.stats(i)["qbits"] for i in imgs)
    rows = sum(i.shape[0] for i in imgs)
    say(f"[gpu] row streams: gap {100 * (got - ideal) / ideal:.4f}% ({(got - ideal) / rows:.2f} bits per row)")
    assert 0.0 <= got - ideal <= 10.0 * rows
    assert (got - ideal) / ideal <= 1e-3


def test_corrupt_rows_detected(models, nx):
    """Damage to a row stream is reported (status 4), never a wrong image
    with status 0; so is a stream table entry pointing past the end."""
    m, _ = models["A"]
    H, W = 70, 40
    img = synth.smooth_field_image(2.0, 3, 0, H, W, 8300)
    t = cuda(img)
    data, offs = m.encode([t], order=nx.WAVEFRONT, interleave=nx.ROWS)
    d = data.cpu().numpy()
    ends = np.frombuffer(bytes(d[32:32 + 4 * H]), dtype="<u4").astype(np.int64)
    pay = 32 + 4 * H
    for r in range(0, H, 3):  # a byte in the middle of every third row's stream
        lo = 0 if r == 0 else int(ends[r - 1])
        mid = pay + (lo + int(ends[r])) // 2
        bad = data.clone()
        bad[mid] ^= 0x5A
        out, st = m.decode(bad, offs, [(H, W)], order=nx.WAVEFRONT, interleave=nx.ROWS, sync=False)
        torch.cuda.synchronize()
        assert int(st[0]) == 4 or torch.equal(out[0], t), r
    bad = data.clone()
    bad[32 + 4 * (H - 1)] ^= 0x7F
    _, st = m.decode(bad, offs, [(H, W)], order=nx.WAVEFRONT, interleave=nx.ROWS, sync=False)
    assert int(st[0]) == 4
    # a container of K streams is not a row-stream container
    d4, o4 = m.encode([t], order=nx.WAVEFRONT, interleave=4)
    _, st = m.decode(d4, o4, [(H, W)], order=nx.WAVEFRONT, interleave=nx.ROWS, sync=False)
    assert int(st[0]) == 4


def test_argument_checks(models, nx):
    m, _ = models["C"]
    t = cuda(np.zeros((8, 8, 3), dtype=np.uint8))
    with pytest.raises(nx.NelloxError):
        m.encode([t], order=nx.RASTER, interleave=nx.ROWS)
    with pytest.raises(nx.NelloxError):
        m.encode([t], order=nx.SHEARED, interleave=nx.ROWS)


def test_prepared_runs_and_static_decode(models, nx):
    """The prepared (capturable) split and the no-allocation entry point
    decode row-stream containers exactly, twice in a row."""
    m, _ = models["B"]
    L = nx.load()
    shapes = [(150, 90), (40, 200)]
    imgs = [synth.smooth_field_image(2.0, 3, 2, H, W, 8400 + k) for k, (H, W) in enumerate(shapes)]
    ts = [cuda(i) for i in imgs]
    data, offs = m.encode(ts, order=nx.WAVEFRONT, interleave=nx.ROWS)
    outs = [torch.zeros_like(x) for x in ts]
    plan, ws = m.decode_prepare(outs, order=nx.WAVEFRONT, interleave=nx.ROWS)
    assert plan.n_bands == 10 + 3  # bands of 16 rows
    # the queue takes the bands by the step they start at: the first band of
    # both images, then the second of both, ...
    order = ws[plan.band_order_offset:plan.band_order_offset + 4 * plan.n_bands].cpu().numpy().view("<i4")
    assert order.tolist() == [0, 10, 1, 11, 2, 12, 3, 4, 5, 6, 7, 8, 9]
    st = torch.empty(2, dtype=torch.int32, device="cuda")
    for _ in range(2):
        for o in outs:
            o.zero_()
        m.decode_run(plan, data, offs, st, ws)
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0 and all(torch.equal(a, b) for a, b in zip(outs, ts))
    for _ in range(2):
        got = [torch.zeros_like(x) for x in ts]
        arr = nx._images(got)
        o = nx._opts(nx.WAVEFRONT, None, nx.ROWS)
        rc = L.nellox_decode_static(m._h, 2, data.data_ptr(), offs.data_ptr(), ctypes.byref(o), arr, st.data_ptr(),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0
        torch.cuda.synchronize()
        assert int(st.abs().sum()) == 0 and all(torch.equal(a, b) for a, b in zip(got, ts))


def test_whole_1024_image(models, nx):
    """One 1024x1024 image, whole-image lane, one stream per row (the paper's
    exact method: no patch borders): exact, with 64 bands pipelined."""
    m, _ = models["B"]
    img = synth.workload_images("large6", count=1)[0]
    t = cuda(img)
    data, offs = m.encode([t], order=nx.WAVEFRONT, interleave=nx.ROWS)
    m.decode(data, offs, [(1024, 1024)], order=nx.WAVEFRONT, interleave=nx.ROWS)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    (out,), st = m.decode(data, offs, [(1024, 1024)], order=nx.WAVEFRONT, interleave=nx.ROWS, sync=False)
    e1.record()
    torch.cuda.synchronize()
    assert int(st[0]) == 0 and torch.equal(out, t)
    say(f"[gpu] whole 1024^2 image, row streams: {e0.elapsed_time(e1):.1f} ms")


def test_band_wait_limit_ends_the_wait(models, nx):
    """The bounded wait on the band above, forced from the host: with a limit
    of one clock tick every band that has to wait gives up at once, marks its
    image corrupt and still finishes (the launch returns); with the default
    limit restored the same container decodes exactly."""
    m, _ = models["C"]
    L = nx.load()
    img = synth.smooth_field_image(2.0, 3, 2, 300, 120, 8500)
    t = cuda(img)
    data, offs = m.encode([t], order=nx.WAVEFRONT, interleave=nx.ROWS)
    prev = L.nellox_debug_band_wait(1)
    try:
        _, st = m.decode(data, offs, [(300, 120)], order=nx.WAVEFRONT, interleave=nx.ROWS, sync=False)
        torch.cuda.synchronize()
        assert int(st[0]) == 4
    finally:
        L.nellox_debug_band_wait(0)
    assert prev == 2_000_000_000
    (out,), st = m.decode(data, offs, [(300, 120)], order=nx.WAVEFRONT, interleave=nx.ROWS)
    assert int(st[0]) == 0 and torch.equal(out, t)


def test_graph_capture_and_replay(models, nx):
    """A prepared row-stream decode captured in a graph (the prep kernel
    clears the band counters, no memset): every replay, with eager work in
    between, decodes exactly, also after other containers of the same shapes
    are copied into the captured input buffers."""
    say("[gpu] row streams, graph capture of a prepared decode")
    m, _ = models["B"]
    shapes = [(150, 90), (40, 200), (33, 17)]
    imgs = [synth.smooth_field_image(2.0, 3, 2, H, W, 8600 + k) for k, (H, W) in enumerate(shapes)]
    ts = [cuda(i) for i in imgs]
    ts2 = [cuda(np.ascontiguousarray(i[::-1, ::-1])) for i in imgs]
    d1, o1 = m.encode(ts, order=nx.WAVEFRONT, interleave=nx.ROWS)
    d2, o2 = m.encode(ts2, order=nx.WAVEFRONT, interleave=nx.ROWS)
    buf = torch.zeros(max(d1.numel(), d2.numel()), dtype=torch.uint8, device="cuda")
    offs = torch.zeros_like(o1)
    buf[:d1.numel()].copy_(d1)
    offs.copy_(o1)
    outs = [torch.zeros_like(t) for t in ts]
    plan, ws = m.decode_prepare(outs, order=nx.WAVEFRONT, interleave=nx.ROWS)
    status = torch.full((len(ts),), 7, dtype=torch.int32, device="cuda")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        m.decode_run(plan, buf, offs, status, ws)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        m.decode_run(plan, buf, offs, status, ws)
    for rep in range(3):
        for o in outs:
            o.zero_()
        status.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(status.abs().sum()) == 0, rep
        assert all(torch.equal(a, b) for a, b in zip(outs, ts)), rep
    buf[:d2.numel()].copy_(d2)
    offs.copy_(o2)
    for rep in range(2):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(status.abs().sum()) == 0
        assert all(torch.equal(a, b) for a, b in zip(outs, ts2))


def test_band_queue_order_with_patches(models, nx):
    """The band order of a batch with patch grids (ragged patch rows, lanes
    of different band counts): a permutation of the bands in which every
    band comes after the one above it in its lane, ordered by band index
    within the lane, then by image and lane (checked against an independent
    enumeration); the batch decodes exactly in that order."""
    m, _ = models["A"]
    shapes = [(100, 70), (37, 50), (70, 33)]
    patch = (40, 32)
    imgs = [synth.smooth_field_image(2.0, 3, 2, H, W, 8700 + k) for k, (H, W) in enumerate(shapes)]
    ts = [cuda(i) for i in imgs]
    data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=nx.ROWS)
    outs = [torch.zeros_like(t) for t in ts]
    plan, ws = m.decode_prepare(outs, order=nx.WAVEFRONT, patch=patch, interleave=nx.ROWS)
    # bands in image order: per image, lanes row-major, a lane's bands in order
    lanes = []  # (image, lane row, lane column, bands)
    base = 0
    bands_of = lambda h: -(-h // 16)  # noqa: E731
    image_order = {}
    for k, (H, W) in enumerate(shapes):
        ph, pw = min(patch[0], H), min(patch[1], W)
        nly, nlx = -(-H // ph), -(-W // pw)
        for ly in range(nly):
            hl = min(ph, H - ly * ph)
            for lx in range(nlx):
                for bb in range(bands_of(hl)):
                    image_order[(k, ly, lx, bb)] = base + ly * nlx * bands_of(ph) + lx * bands_of(hl) + bb
        base += (nly - 1) * nlx * bands_of(ph) + nlx * bands_of(H - (nly - 1) * ph)
    assert plan.n_bands == base == len(image_order)
    want = [image_order[key] for key in sorted(image_order, key=lambda t: (t[3], t[0], t[1], t[2]))]
    got = ws[plan.band_order_offset:plan.band_order_offset + 4 * plan.n_bands].cpu().numpy().view("<i4").tolist()
    assert got == want
    st = torch.empty(len(ts), dtype=torch.int32, device="cuda")
    m.decode_run(plan, data, offs, st, ws)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0 and all(torch.equal(a, b) for a, b in zip(outs, ts))
