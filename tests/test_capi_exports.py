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
    # bad blobs are rejected before any device call
    h = ctypes.c_void_p()
    assert L.nellox_model_create(b"NLXWxxxx", 8, ctypes.byref(h)) == 2
    assert b"blob" in L.nellox_last_error()
    hdr = bytearray(32)
    hdr[0:4] = b"NLXC"
    hdr[4], hdr[5], hdr[6], hdr[7] = 1, 1, 3, 1
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


def test_product_has_no_cpu_fallback():
    # the binding imports only the HIP library; the oracle is test-only
    src = open(os.path.join(ROOT, "paper_2201_05213_amd", "__init__.py")).read()
    src += open(os.path.join(ROOT, "paper_2201_05213_amd", "_lib.py")).read()
    assert "oracle" not in src and "synth" not in src
