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

__all__ = ["autotune"]


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
