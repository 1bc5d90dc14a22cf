"""The no-allocation decoder (nellox_decode_static, through the C ABI)
against nellox_decode with a caller's workspace: the same images and the same
status, on two calls in a row, the second with a smaller batch (the scratch
array keeps the first call's contents), in the wavefront, sheared and raster
orders; and a batch beyond the scratch is refused before any launch."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import paper_2201_05213_amd as nx

    torch.cuda.set_device(0)
    return nx, nx.Model(synth.model_blob("B")[0])


def decode_static(nx, m, data, offs, shapes, order, patch, K):
    L = nx.load()
    outs = [torch.full((h, w, 3), 7, dtype=torch.uint8, device="cuda") for h, w in shapes]
    arr = nx._images(outs)
    st = torch.full((len(shapes),), -1, dtype=torch.int32, device="cuda")
    o = nx._opts(order, patch, K)
    rc = L.nellox_decode_static(m._h, len(shapes), data.data_ptr(), offs.data_ptr(), ctypes.byref(o), arr,
                                st.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, L.nellox_last_error()
    torch.cuda.synchronize()
    return outs, st


@pytest.mark.parametrize("order,patch,K", [(1, (64, 64), 4), (2, (86, 64), 4), (2, None, 1), (0, None, 1)])
def test_static_decode_matches_workspace_decode(setup, order, patch, K):
    nx, m = setup
    big = [synth.smooth_field_image(4.0, 20, 3, 300, 260, 7000 + k) for k in range(3)]
    small = [synth.smooth_field_image(2.0, 3, 0, 40, 70, 7100)]
    if order == 0:
        big = [b[:40, :90].copy() for b in big[:2]]
    for imgs in (big, small):  # the second call is smaller than the first
        say(f"[gpu] static decode order {order} patch {patch} K {K}: {len(imgs)} images {imgs[0].shape}")
        ts = [torch.from_numpy(i).cuda() for i in imgs]
        shapes = [i.shape[:2] for i in imgs]
        data, offs = m.encode(ts, order=1 if order == 2 else order, patch=patch, interleave=K)
        ref, rst = m.decode(data, offs, shapes, order=order, patch=patch, interleave=K, sync=False)
        got, gst = decode_static(nx, m, data, offs, shapes, order, patch, K)
        assert torch.equal(gst, rst) and int(gst.abs().sum()) == 0
        for a, b, t in zip(got, ref, ts):
            assert torch.equal(a, b) and torch.equal(a, t)


def test_static_decode_refuses_oversized_batch(setup):
    nx, m = setup
    L = nx.load()
    # 3000 descriptors exceed the plan staging; refused on the host, nothing launched
    shapes = [(8, 8)] * 3000
    arr = (nx._lib.NelloxImage * len(shapes))(*[nx._lib.NelloxImage(1, h, w) for h, w in shapes])
    o = nx._opts(1, None, 1)
    rc = L.nellox_decode_static(m._h, len(shapes), 1, 1, ctypes.byref(o), arr, 1, None)
    assert rc == 3 and b"images per call" in L.nellox_last_error()
    # sheared windows of many tall lanes exceed the 32 MiB scratch
    shapes = [(65535, 1024)] * 2
    arr = (nx._lib.NelloxImage * 2)(*[nx._lib.NelloxImage(1, h, w) for h, w in shapes])
    o = nx._opts(2, (65535, 4), 1)
    need = L.nellox_decode_workspace_bytes(m._h, 2, arr, ctypes.byref(o))
    assert need > 32 << 20
    rc = L.nellox_decode_static(m._h, 2, 1, 1, ctypes.byref(o), arr, 1, None)
    assert rc == 3 and b"no-allocation decoder" in L.nellox_last_error()
