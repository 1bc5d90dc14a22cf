"""FP64 CPU oracle: ctypes binding of nellox_oracle.c plus a torch-FP64 reference.

TEST INFRASTRUCTURE ONLY. The product (the HIP library and its Python
binding) never imports this package; only tests, the smoke check and the
benchmark's CPU-baseline leg do. It shares no code with the GPU path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nellox_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

E_NAN = -5
E_CDF = -6
E_CORRUPT = -4


def build() -> str:
    """Compile the oracle with gcc (plain C99, -O2)."""
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P, I, D, L64, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_long, ctypes.c_size_t
        L.ox_model_new.restype = P
        L.ox_model_new.argtypes = [I, I, I, P]
        L.ox_model_from_blob.restype = P
        L.ox_model_from_blob.argtypes = [P, S, P, P]
        L.ox_model_free.argtypes = [P]
        L.ox_param_count.restype = L64
        L.ox_param_count.argtypes = [I, I, I]
        L.ox_stats.restype = I
        L.ox_stats.argtypes = [P, P, I, I, I, I, P, P, P]
        L.ox_theta_image.restype = I
        L.ox_theta_image.argtypes = [P, P, I, I, P]
        L.ox_encode.restype = L64
        L.ox_encode.argtypes = [P, P, I, I, I, I, I, P, S]
        L.ox_decode.restype = I
        L.ox_decode.argtypes = [P, P, S, I, I, I, I, I, P]
        L.ox_rans_encode.restype = L64
        L.ox_rans_encode.argtypes = [P, P, L64, P, S]
        L.ox_rans_decode.restype = L64
        L.ox_rans_decode.argtypes = [P, L64, P, S, P]
        L.ox_spread_select.restype = ctypes.c_uint32
        L.ox_spread_select.argtypes = [ctypes.c_uint32] * 3
        L.ox_spread_rank.restype = ctypes.c_uint32
        L.ox_spread_rank.argtypes = [ctypes.c_uint32] * 3
        L.ox_encode_offset.restype = L64
        L.ox_encode_offset.argtypes = [P, P, I, I, I, I, I, P, S]
        L.ox_decode_offset.restype = I
        L.ox_decode_offset.argtypes = [P, P, S, I, I, I, I, I, P]
        L.ox_symbol_order.restype = L64
        L.ox_symbol_order.argtypes = [I, I, I, P]
        L.ox_tap_live.restype = I
        L.ox_tap_live.argtypes = [I, I, I]
        L.ox_steps.restype = L64
        L.ox_steps.argtypes = [I, I, I]
        L.ox_lane_count.restype = I
        L.ox_lane_count.argtypes = [I, I, I, I]
        L.ox_log_bin.restype = D
        L.ox_log_bin.argtypes = [I, D, D]
        L.ox_shear.restype = None
        L.ox_shear.argtypes = [P, I, I, I, I, P]
        L.ox_unshear.restype = None
        L.ox_unshear.argtypes = [P, I, I, I, I, P]
        L.ox_shear_tap_live.restype = I
        L.ox_shear_tap_live.argtypes = [I, I, I]
        L.ox_shear_kernel.restype = None
        L.ox_shear_kernel.argtypes = [P, P]
        L.ox_theta_image_shear.restype = I
        L.ox_theta_image_shear.argtypes = [P, P, I, I, P]
        L.ox_decode_shear.restype = I
        L.ox_decode_shear.argtypes = [P, P, S, I, I, I, I, P]
        L.ox_philox4x64.restype = None
        L.ox_philox4x64.argtypes = [P, P, P]
        L.ox_sample_slot.restype = ctypes.c_uint32
        L.ox_sample_slot.argtypes = [ctypes.c_uint64, I, I, I, I]
        L.ox_sample.restype = I
        L.ox_sample.argtypes = [P, I, I, I, I, I, ctypes.c_uint64, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


class Model:
    """An FP64 oracle model (its own copy of the parameters, double precision)."""

    def __init__(self, handle, dims):
        self._h = handle
        self.h, self.C, self.n_blocks = dims

    @classmethod
    def from_blob(cls, blob: bytes) -> "Model":
        L = lib()
        dims = np.zeros(3, dtype=np.int32)
        hsh = np.zeros(1, dtype=np.uint64)
        buf = np.frombuffer(blob, dtype=np.uint8).copy()
        h = L.ox_model_from_blob(_ptr(buf), buf.size, _ptr(dims), _ptr(hsh))
        if not h:
            raise ValueError("oracle rejected the weight blob")
        m = cls(h, tuple(int(x) for x in dims))
        m.hash = int(hsh[0])
        return m

    @classmethod
    def from_params(cls, h: int, C: int, n_blocks: int, params) -> "Model":
        L = lib()
        p = np.ascontiguousarray(params, dtype=np.float64)
        if p.size != L.ox_param_count(h, C, n_blocks):
            raise ValueError("parameter count does not match dims")
        hd = L.ox_model_new(h, C, n_blocks, _ptr(p))
        if not hd:
            raise ValueError("bad dims")
        return cls(hd, (h, C, n_blocks))

    def __del__(self):
        try:
            if self._h:
                lib().ox_model_free(self._h)
        except Exception:
            pass

    # -- statistics -------------------------------------------------------
    def stats(self, img: np.ndarray, ph: int = 0, pw: int = 0, cdf: bool = False, px_bits: bool = False):
        """Returns dict(qbits, cbits[, cdf (H,W,3,257) int32][, px_bits (H,W)])."""
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W, _ = img.shape
        out = np.zeros(2, dtype=np.float64)
        cd = np.zeros((H, W, 3, 257), dtype=np.int32) if cdf else None
        pb = np.zeros((H, W), dtype=np.float64) if px_bits else None
        rc = lib().ox_stats(self._h, _ptr(img), H, W, ph, pw, _ptr(out),
                            _ptr(cd) if cd is not None else None, _ptr(pb) if pb is not None else None)
        if rc:
            raise OracleError(rc, "stats")
        r = dict(qbits=float(out[0]), cbits=float(out[1]))
        if cd is not None:
            r["cdf"] = cd
        if pb is not None:
            r["px_bits"] = pb
        return r

    def theta_image(self, img: np.ndarray) -> np.ndarray:
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W, _ = img.shape
        th = np.zeros((H, W, 100), dtype=np.float64)
        rc = lib().ox_theta_image(self._h, _ptr(img), H, W, _ptr(th))
        if rc:
            raise OracleError(rc, "theta")
        return th

    # -- codec ------------------------------------------------------------
    def encode(self, img: np.ndarray, order: int = 0, ph: int = 0, pw: int = 0,
               offset: int | None = None) -> bytes:
        """order 0 raster, 1 wavefront (step j + (h+1) i); `offset` overrides
        the wavefront step offset (tests of non-causal orders)."""
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W, _ = img.shape
        cap = 64 + 8 * H * W * 3 + 16 * lib().ox_lane_count(H, W, ph, pw)
        out = np.zeros(cap, dtype=np.uint8)
        if offset is None:
            offset = (self.h + 1) if order == 1 else 0
        n = lib().ox_encode_offset(self._h, _ptr(img), H, W, offset, ph, pw, _ptr(out), cap)
        if n < 0:
            raise OracleError(n, "encode")
        return out[:n].tobytes()

    def decode(self, data: bytes, H: int, W: int, order: int = 0, ph: int = 0, pw: int = 0,
               offset: int | None = None) -> np.ndarray:
        buf = np.frombuffer(data, dtype=np.uint8).copy()
        img = np.zeros((H, W, 3), dtype=np.uint8)
        if offset is None:
            offset = (self.h + 1) if order == 1 else 0
        rc = lib().ox_decode_offset(self._h, _ptr(buf), buf.size, H, W, offset, ph, pw, _ptr(img))
        if rc:
            raise OracleError(rc, "decode")
        return img


    # -- ShearLoC (Sec. 3.1, Algorithm 2) -----------------------------------
    def shear_kernel(self) -> np.ndarray:
        """The sheared first kernel, (C, 3, h+1, h(h+2))."""
        h = self.h
        Kp = np.zeros((self.C, 3, h + 1, h * (h + 2)), dtype=np.float64)
        lib().ox_shear_kernel(self._h, _ptr(Kp))
        return Kp

    def theta_image_shear(self, img: np.ndarray) -> np.ndarray:
        img = np.ascontiguousarray(img, dtype=np.uint8)
        H, W, _ = img.shape
        th = np.zeros((H, W, 100), dtype=np.float64)
        rc = lib().ox_theta_image_shear(self._h, _ptr(img), H, W, _ptr(th))
        if rc:
            raise OracleError(rc, "theta_shear")
        return th

    def decode_shear(self, data: bytes, H: int, W: int, ph: int = 0, pw: int = 0) -> np.ndarray:
        """Decode a wavefront-order container with the sheared model."""
        buf = np.frombuffer(data, dtype=np.uint8).copy()
        img = np.zeros((H, W, 3), dtype=np.uint8)
        rc = lib().ox_decode_shear(self._h, _ptr(buf), buf.size, H, W, ph, pw, _ptr(img))
        if rc:
            raise OracleError(rc, "decode_shear")
        return img

    # -- sampling ---------------------------------------------------------
    def sample(self, H: int, W: int, seed: int, order: int = 1, ph: int = 0, pw: int = 0,
               offset: int | None = None) -> np.ndarray:
        """Ancestral sample (H, W, 3) uint8: each symbol is the inverse
        quantised CDF at its Philox slot (see sample_slots)."""
        img = np.zeros((H, W, 3), dtype=np.uint8)
        if offset is None:
            offset = (self.h + 1) if order == 1 else 0
        rc = lib().ox_sample(self._h, H, W, offset, ph, pw, seed, _ptr(img))
        if rc:
            raise OracleError(rc, "sample")
        return img


def shear(x: np.ndarray, o: int) -> np.ndarray:
    """(H, W[, nc]) -> (H, W + o (H - 1)[, nc]) sheared with offset o."""
    a = np.ascontiguousarray(x, dtype=np.float64)
    squeeze = a.ndim == 2
    if squeeze:
        a = a[:, :, None]
    H, W, nc = a.shape
    S = np.zeros((H, W + o * (H - 1), nc), dtype=np.float64)
    lib().ox_shear(_ptr(a), H, W, nc, o, _ptr(S))
    return S[:, :, 0] if squeeze else S


def unshear(S: np.ndarray, W: int, o: int) -> np.ndarray:
    a = np.ascontiguousarray(S, dtype=np.float64)
    squeeze = a.ndim == 2
    if squeeze:
        a = a[:, :, None]
    H, _, nc = a.shape
    x = np.zeros((H, W, nc), dtype=np.float64)
    lib().ox_unshear(_ptr(a), H, W, nc, o, _ptr(x))
    return x[:, :, 0] if squeeze else x


def shear_tap_live(h: int, a: int, q: int) -> bool:
    return bool(lib().ox_shear_tap_live(h, a, q))


def philox4x64(ctr, key) -> np.ndarray:
    """One Philox4x64-10 block: 4 uint64 from a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    lib().ox_philox4x64(_ptr(c), _ptr(k), _ptr(o))
    return o


def sample_slot(seed: int, W: int, y: int, x: int, c: int) -> int:
    return int(lib().ox_sample_slot(seed, W, y, x, c))


def rans_encode(start, freq) -> bytes:
    s = np.ascontiguousarray(start, dtype=np.uint32)
    f = np.ascontiguousarray(freq, dtype=np.uint32)
    cap = 8 + 2 * s.size + 16
    out = np.zeros(cap, dtype=np.uint8)
    n = lib().ox_rans_encode(_ptr(s), _ptr(f), s.size, _ptr(out), cap)
    if n < 0:
        raise OracleError(n, "rans_encode")
    return out[:n].tobytes()


def spread_select(x: int, start: int, freq: int) -> int:
    """The x-th (from 0) slot y in [0, 2^16) whose 16-bit reversal lies in
    [start, start + freq): where the coder puts a push from a state x < freq."""
    return int(lib().ox_spread_select(x, start, freq))


def spread_rank(y: int, start: int, freq: int) -> int:
    """Number of spread slots of (start, freq) below y."""
    return int(lib().ox_spread_rank(y, start, freq))


def rans_decode(cdfs: np.ndarray, data: bytes):
    """cdfs: (N, 257) int32 rows; returns (symbols, ok)."""
    c = np.ascontiguousarray(cdfs, dtype=np.int32)
    N = c.shape[0]
    buf = np.frombuffer(data, dtype=np.uint8).copy() if len(data) else np.zeros(1, dtype=np.uint8)
    sym = np.zeros(N, dtype=np.int32)
    rc = lib().ox_rans_decode(_ptr(c), N, _ptr(buf), len(data), _ptr(sym))
    return sym, rc == 0


def symbol_order(H: int, W: int, offset: int) -> np.ndarray:
    """Decode order of a lane as an (N, 3) array of (i, j, channel)."""
    seq = np.zeros((3 * H * W, 3), dtype=np.int32)
    n = lib().ox_symbol_order(H, W, offset, _ptr(seq))
    return seq[:n]


def tap_live(h: int, dy: int, dx: int) -> bool:
    return bool(lib().ox_tap_live(h, dy, dx))


def steps(H: int, W: int, h: int) -> int:
    return int(lib().ox_steps(H, W, h))


def log_bin(k: int, mu: float, invs: float) -> float:
    return float(lib().ox_log_bin(k, mu, invs))
