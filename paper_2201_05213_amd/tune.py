"""Autotuning of the coding layout for a batch: patch shape and rANS streams
per lane (opts.patch_*, opts.interleave).

Smaller patches give the decoder more independent lanes (more waves per CU)
but fewer pixels per wavefront step and more bits (context lost at patch
borders); more streams per lane cost one stream flush each. The tuner encodes
the batch with every candidate, times the decode (prepared, kernels only,
median of `reps`), and picks the fastest candidate whose coded bits are within
`max_bits_cost` (relative) of the fewest bits any candidate reached.
"""
from __future__ import annotations

import statistics

import torch

from . import WAVEFRONT, payload_bits

__all__ = ["autotune", "balanced_patch", "lane_count"]

SIMDS_PER_CU = 4


def lane_count(shapes, patch) -> int:
    """Lanes of a batch of (H, W) images cut into patch = (rows, cols) tiles."""
    ph, pw = patch
    return sum(-(-int(H) // ph) * -(-int(W) // pw) for H, W in shapes)


def balanced_patch(shapes, cols: int = 64, cus: int | None = None, lanes_per_simd: int = 2, min_rows: int = 64,
                   min_tail: float = 0.5):
    """The shortest patch (rows, cols) that puts at most `lanes_per_simd`
    lanes on any SIMD of the decoder's launch.

    A lane is one wave, and when every lane of a batch fits in the launch at
    once the decode takes as long as the busiest SIMD's lanes, back to back:
    its FP32 MFMA and VALU issue do not overlap across waves. One wave per
    SIMD leaves it latency-bound, two fill it; so the fastest layout is the
    shortest lane for which the batch needs at most two waves per SIMD. With
    64 columns a lane's 16-row group is full (64 / (h + 1) rows per step for
    h = 3). Heights below `min_rows` are not considered (every rANS stream
    costs ~16 bits, so short lanes cost bits), nor heights whose last lane row
    of some image is shorter than `min_tail` of the patch (a thin ragged lane
    pays the same per-stream cost for few pixels)."""
    if cus is None:
        import torch

        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    cap = lanes_per_simd * SIMDS_PER_CU * int(cus)
    tallest = max(int(H) for H, _ in shapes)
    for ph in range(min_rows, max(tallest, min_rows) + 1):
        if lane_count(shapes, (ph, cols)) > cap:
            continue
        tails = [int(H) - (-(-int(H) // ph) - 1) * ph for H, _ in shapes if int(H) > ph]
        if all(t >= min_tail * ph for t in tails):
            return ph, cols
    return max(tallest, min_rows), cols


def autotune(model, imgs, patches=((32, 32), (64, 64)), interleaves=(1, 2, 4), max_bits_cost: float = 1e-3,
             reps: int = 3):
    """Returns (choice, table): dicts with keys patch, interleave, decode_ms,
    bits; `choice` is the selected row of `table`."""
    table = []
    stream = torch.cuda.current_stream(model.device)
    for patch in patches:
        for K in interleaves:
            data, offs = model.encode(imgs, order=WAVEFRONT, patch=patch, interleave=K)
            bits = sum(payload_bits(data, offs))
            out = [torch.empty_like(t) for t in imgs]
            plan, ws = model.decode_prepare(out, order=WAVEFRONT, patch=patch, interleave=K)
            status = torch.empty(max(len(imgs), 1), dtype=torch.int32, device=model.device)
            model.decode_run(plan, data, offs, status, ws)
            times = []
            for _ in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                model.decode_run(plan, data, offs, status, ws)
                b.record(stream)
                b.synchronize()
                times.append(a.elapsed_time(b))
            if int(status.abs().sum()) != 0 or not all(torch.equal(x, y) for x, y in zip(out, imgs)):
                raise RuntimeError(f"decode check failed for patch {patch}, interleave {K}")
            table.append({"patch": tuple(patch), "interleave": K, "decode_ms": statistics.median(times),
                          "bits": bits})
    best = min(r["bits"] for r in table)
    ok = [r for r in table if r["bits"] <= best * (1.0 + max_bits_cost)]
    choice = min(ok, key=lambda r: r["decode_ms"])
    return choice, table
