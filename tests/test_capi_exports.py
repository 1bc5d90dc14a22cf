"""CPU checks of the boundary: the HIP library loads and exports every entry
point include/nellox.h declares (no compute calls: no GPU here), and the
host-only calls behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nellox.h")
LIB = os.path.join(ROOT, "paper_2201_05213_amd", "libnellox.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nellox_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnellox.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_api():
    names = declared()
    for n in ("nellox_model_create", "nellox_encode", "nellox_decode", "nellox_nll", "nellox_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_2201_05213_amd import _lib

    assert sorted(_lib.SIGNATURES) == declared()


def test_host_only_calls(lib):
    from paper_2201_05213_amd import _lib

    L = _lib.load()
    o = _lib.NelloxOpts(1, 64, 64, 0)
    # header + lane table + 4 flush bytes per lane + 2 bytes per symbol
    assert L.nellox_encode_bound(128, 128, ctypes.byref(o)) == 32 + 4 * 4 + 4 * 4 + 6 * 128 * 128
    assert L.nellox_encode_bound(0, 5, ctypes.byref(o)) == 0
    o2 = _lib.NelloxOpts(1, 64, 64, 2)
    assert L.nellox_encode_bound(128, 128, ctypes.byref(o2)) == 32 + 4 * 4 * 2 + 4 * 4 * 2 + 6 * 128 * 128
    assert L.nellox_encode_bound(128, 128, ctypes.byref(_lib.NelloxOpts(1, 64, 64, 3))) == 0
    # bad blobs are rejected before any device call
    h = ctypes.c_void_p()
    assert L.nellox_model_create(b"NLXWxxxx", 8, ctypes.byref(h)) == 2
    assert b"blob" in L.nellox_last_error()
    hdr = bytearray(32)
    hdr[0:4] = b"NLXC"
    hdr[4], hdr[5], hdr[6], hdr[7] = 2, 1, 3, 1  # container version 2
    hdr[8:12] = (200).to_bytes(4, "little")
    hdr[12:16] = (320).to_bytes(4, "little")
    hdr[16:18] = (64).to_bytes(2, "little")
    hdr[18:20] = (32).to_bytes(2, "little")
    H, W = ctypes.c_int32(), ctypes.c_int32()
    oo = _lib.NelloxOpts()
    buf = ctypes.create_string_buffer(bytes(hdr), 32)
    assert L.nellox_peek(buf, 32, ctypes.byref(H), ctypes.byref(W), ctypes.byref(oo)) == 0
    assert (H.value, W.value, oo.order, oo.patch_h, oo.patch_w) == (200, 320, 1, 64, 32)
    assert L.nellox_peek(buf, 31, ctypes.byref(H), ctypes.byref(W), ctypes.byref(oo)) == 4
    # containers of the first format (start state 1 by ranges, four flush bytes) are refused
    hdr[4] = 1
    buf1 = ctypes.create_string_buffer(bytes(hdr), 32)
    assert L.nellox_peek(buf1, 32, ctypes.byref(H), ctypes.byref(W), ctypes.byref(oo)) == 4


def test_training_host_calls(lib):
    from paper_2201_05213_amd import _lib, blob

    L = _lib.load()
    for h, C, nb in [(3, 64, 2), (3, 32, 1), (2, 32, 1), (3, 8, 1), (1, 16, 0)]:
        d = (ctypes.c_int32 * 4)(h, C, nb, 10)
        assert L.nellox_param_count(d) == blob.param_count(h, C, nb)
        assert L.nellox_train_workspace_bytes(d, 4, 32, 32) > 4 * 4 * 32 * 32 * (3 * (2 * nb + 1) * C)
    for bad in [(0, 32, 1, 10), (3, 32, 1, 9), (4, 16, 0, 10)]:
        d = (ctypes.c_int32 * 4)(*bad)
        assert L.nellox_param_count(d) == -1 or bad[0] == 4
        assert L.nellox_train_workspace_bytes(d, 4, 32, 32) == 0
    d = (ctypes.c_int32 * 4)(3, 64, 2, 10)
    assert L.nellox_train_workspace_bytes(d, 0, 32, 32) == 0
    assert L.nellox_train_workspace_bytes(d, 4, 0, 32) == 0


def test_blob_round_trip():
    import synth
    from paper_2201_05213_amd import blob

    for name in ("A", "B", "C", "tiny"):
        b, dims = synth.model_blob(name)
        d, p = blob.params_from_blob(b)
        assert d == (dims["h"], dims["C"], dims["n_blocks"], 10)
        assert blob.blob_from_params(d, p) == b
    b, _ = synth.model_blob("tiny")
    with pytest.raises(ValueError):
        blob.params_from_blob(b[:-1] + bytes([b[-1] ^ 1]))


def test_product_has_no_cpu_fallback():
    # the binding imports only the HIP library; the oracle is test-only
    src = ""
    for f in ("__init__.py", "_lib.py", "train.py", "blob.py"):
        src += open(os.path.join(ROOT, "paper_2201_05213_amd", f)).read()
    assert "oracle" not in src and "synth" not in src
