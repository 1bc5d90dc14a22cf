"""Seeded random weights and the weight-blob byte format.

Blob layout (little endian):
  b"NLXW", u32 version (=1), u32 h, u32 C, u32 n_blocks, u32 n_mix (=10),
  u32 flags (=1: channel posteriors conditioned on earlier channels)
  FP32 tensors, in this order:
    conv_w [C][3][2h+1][2h+1], conv_b [C],
    per residual block: w1 [C][C], b1 [C], w2 [C][C], b2 [C],
    head_w [10*n_mix][C], head_b [10*n_mix]
  u64 FNV-1a (64-bit) of every preceding byte.

The first kernel is stored dense; readers use only its causal taps, so the
generator fills every position (a reader that forgets the mask then leaks
future pixels, which the tests detect).
"""
from __future__ import annotations

import struct

import numpy as np

BLOB_MAGIC = b"NLXW"
BLOB_VERSION = 1

# (h, C, n_blocks) of the named models and their weight seeds
MODEL_DIMS = {
    "A": dict(h=3, C=32, n_blocks=1, seed=11),
    "B": dict(h=3, C=64, n_blocks=2, seed=12),
    "C": dict(h=2, C=32, n_blocks=1, seed=13),
    "tiny": dict(h=3, C=8, n_blocks=1, seed=14),
}


def param_shapes(h: int, C: int, n_blocks: int, n_mix: int = 10):
    K = 2 * h + 1
    shapes = [("conv_w", (C, 3, K, K)), ("conv_b", (C,))]
    for b in range(n_blocks):
        shapes += [(f"w1_{b}", (C, C)), (f"b1_{b}", (C,)), (f"w2_{b}", (C, C)), (f"b2_{b}", (C,))]
    shapes += [("head_w", (10 * n_mix, C)), ("head_b", (10 * n_mix,))]
    return shapes


def param_count(h: int, C: int, n_blocks: int, n_mix: int = 10) -> int:
    return int(sum(int(np.prod(s)) for _, s in param_shapes(h, C, n_blocks, n_mix)))


def init_params(h: int, C: int, n_blocks: int, seed: int, n_mix: int = 10) -> np.ndarray:
    """Flat FP32 parameter vector, U(+-1/sqrt(fan_in)) for weights and biases.

    fan_in is 3*(2h+1)^2 for the first layer and C for the 1x1 layers.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    K = 2 * h + 1
    out = []
    for name, shape in param_shapes(h, C, n_blocks, n_mix):
        fan_in = 3 * K * K if name.startswith("conv") else C
        bound = 1.0 / np.sqrt(fan_in)
        out.append(rng.uniform(-bound, bound, size=int(np.prod(shape))))
    return np.concatenate(out).astype(np.float32)


def fnv1a64(data: bytes) -> int:
    h = 0xCBF29CE484222325
    for b in data:
        h ^= b
        h = (h * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


def write_blob(h: int, C: int, n_blocks: int, params: np.ndarray, n_mix: int = 10,
               flags: int = 1) -> bytes:
    params = np.ascontiguousarray(params, dtype="<f4")
    if params.size != param_count(h, C, n_blocks, n_mix):
        raise ValueError("parameter count does not match dims")
    head = BLOB_MAGIC + struct.pack("<6I", BLOB_VERSION, h, C, n_blocks, n_mix, flags)
    body = head + params.tobytes()
    return body + struct.pack("<Q", fnv1a64(body))


def model_blob(name: str) -> tuple[bytes, dict]:
    d = MODEL_DIMS[name]
    p = init_params(d["h"], d["C"], d["n_blocks"], d["seed"])
    return write_blob(d["h"], d["C"], d["n_blocks"], p), dict(d)


def delta_params(h: int, C: int, means=(-100.0, 100.0, -100.0)) -> np.ndarray:
    """A model with no blocks whose every conditional is the same mixture: all
    weights zero; the head bias gives component 0 logit 100 (the others 0),
    mean means[c] to every component of channel c, log-scale -7 and zero
    coefficients. A mean far below -1 puts all of F's mass into bin 0 (and
    far above 1 into bin 255), so the quantised CDF is known in closed form."""
    p = np.zeros(param_count(h, C, 0), dtype=np.float32)
    hb = p[-100:]
    hb[0] = 100.0
    for c in range(3):
        hb[10 + 10 * c:20 + 10 * c] = means[c]
        hb[40 + 10 * c:50 + 10 * c] = -7.0
    return p
