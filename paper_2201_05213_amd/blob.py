"""Weight blob <-> flat parameter vector (the format nellox_model_create reads).

Layout (little endian): b"NLXW", u32 version 1, u32 h, u32 C, u32 n_blocks,
u32 n_mix = 10, u32 flags = 1 (channel weights are posteriors given the
earlier channels), the FP32 tensors conv_w[C][3][2h+1][2h+1], conv_b[C],
per block w1[C][C], b1[C], w2[C][C], b2[C], head_w[100][C], head_b[100],
then the u64 FNV-1a hash of every preceding byte.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"NLXW"
VERSION = 1
_FNV_OFFSET = 0xCBF29CE484222325
_FNV_PRIME = 0x100000001B3


def fnv1a64(data: bytes) -> int:
    h = _FNV_OFFSET
    for b in data:
        h = ((h ^ b) * _FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def param_count(h: int, C: int, n_blocks: int) -> int:
    K = 2 * h + 1
    return C * 3 * K * K + C + n_blocks * (2 * C * C + 2 * C) + 100 * C + 100


def blob_from_params(dims, params) -> bytes:
    h, C, nb, n_mix = (int(v) for v in dims)
    p = np.ascontiguousarray(np.asarray(params, dtype="<f4"))
    if n_mix != 10 or p.size != param_count(h, C, nb):
        raise ValueError("parameter vector does not match dims")
    body = MAGIC + struct.pack("<6I", VERSION, h, C, nb, n_mix, 1) + p.tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


def params_from_blob(blob: bytes):
    """-> (dims (h, C, n_blocks, 10), float32 parameter vector)."""
    if len(blob) < 40 or blob[:4] != MAGIC:
        raise ValueError("not a weight blob")
    ver, h, C, nb, n_mix, _flags = struct.unpack_from("<6I", blob, 4)
    if ver != VERSION or n_mix != 10:
        raise ValueError("unsupported blob version or mixture size")
    n = param_count(h, C, nb)
    if len(blob) != 28 + 4 * n + 8:
        raise ValueError("blob size does not match its dims")
    if struct.unpack_from("<Q", blob, 28 + 4 * n)[0] != fnv1a64(blob[:28 + 4 * n]):
        raise ValueError("blob hash mismatch")
    return (h, C, nb, n_mix), np.frombuffer(blob, dtype="<f4", count=n, offset=28).astype(np.float32)
