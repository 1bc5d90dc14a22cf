"""Autotuning of the coding layout for a batch: patch shape and rANS streams
per lane (opts.patch_*, opts.interleave).

Smaller patches give the decoder more independent lanes (more waves per CU)
but fewer pixels per wavefront step and more bits (context lost at patch
borders); more streams per lane cost a few bits each (the flush's rounding to
whole bytes, under 5 bits on average). The tuner encodes the batch with every
candidate, times the decode (prepared, kernels only, median of `reps`), and
picks the fastest candidate that passes two bits checks: its coded bits are
within `max_bits_cost` (relative) of the reference bits (whole-image coding,
the paper's own layout, or the fewest bits any candidate reached), and the
streams of every image cost at most `max_bits_cost` of that image's bits.
"""
from __future__ import annotations

import statistics

import torch

from . import ROWS, WAVEFRONT, payload_bits

__all__ = ["autotune", "balanced_patch", "lane_count", "image_streams", "STREAM_BITS"]

SIMDS_PER_CU = 4

# mean cost of one rANS stream in bits (start state and the flush rounded to
# whole bytes); the coder's measured mean is ~4.6 bits, its pinned bound 5
STREAM_BITS = 5.0


def lane_count(shapes, patch) -> int:
    """Lanes of a batch of (H, W) images cut into patch = (rows, cols) tiles."""
    ph, pw = patch
    return sum(-(-int(H) // ph) * -(-int(W) // pw) for H, W in shapes)


def image_streams(H: int, W: int, patch, interleave: int) -> int:
    """rANS streams of one H x W image: K per lane, or one per lane row with
    row streams (interleave ROWS); patch None is one whole-image lane."""
    ph, pw = (H, W) if patch is None else (min(patch[0], H), min(patch[1], W))
    nly, nlx = -(-H // ph), -(-W // pw)
    if interleave == ROWS:
        return nlx * H
    return nlx * nly * interleave


def balanced_patch(shapes, cols: int = 64, cus: int | None = None, lanes_per_simd: int = 2, min_rows: int = 64,
                   min_tail: float = 0.25, interleave: int = 1, bits_per_dim: float | None = None,
                   max_bits_cost: float = 1e-3):
    """The shortest patch (rows, cols) that puts at most `lanes_per_simd`
    lanes on any SIMD of the decoder's launch.

    A lane is one wave, and when every lane of a batch fits in the launch at
    once the decode takes as long as the busiest SIMD's lanes, back to back:
    its FP32 MFMA and VALU issue do not overlap across waves. One wave per
    SIMD leaves it latency-bound, two fill it; so the fastest layout is the
    shortest lane for which the batch needs at most two waves per SIMD. With
    64 columns a lane's 16-row group is full (64 / (h + 1) rows per step for
    h = 3). Heights below `min_rows` are not considered, nor heights whose
    last lane row of some image is shorter than `min_tail` of the patch (a
    thin ragged lane pays the same stream cost for few pixels; with ~5 bits
    per stream a quarter of a lane keeps it small). Given the expected
    `bits_per_dim`, heights whose full lane's `interleave` streams cost more
    than `max_bits_cost` of the lane's bits are not considered either."""
    if cus is None:
        import torch

        cus = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    cap = lanes_per_simd * SIMDS_PER_CU * int(cus)
    tallest = max(int(H) for H, _ in shapes)
    for ph in range(min_rows, max(tallest, min_rows) + 1):
        if lane_count(shapes, (ph, cols)) > cap:
            continue
        if bits_per_dim is not None and interleave * STREAM_BITS > max_bits_cost * 3 * ph * cols * bits_per_dim:
            continue
        tails = [int(H) - (-(-int(H) // ph) - 1) * ph for H, _ in shapes if int(H) > ph]
        if all(t >= min_tail * ph for t in tails):
            return ph, cols
    return max(tallest, min_rows), cols


def autotune(model, imgs, patches=(None, (32, 32), (64, 64)), interleaves=(1, 2, 4, 8, 16), rows: bool = True,
             reference: str = "whole", max_bits_cost: float = 1e-3, reps: int = 3):
    """Returns (choice, table): dicts with keys patch, interleave, decode_ms,
    bits, stream_cost (the largest share of an image's bits its streams
    cost), ok; `choice` is the selected row of `table`.

    Candidates are every patch (None: whole-image lanes) with every number of
    interleaved streams, and, if `rows`, whole-image lanes with one stream per
    row (interleave ROWS). `reference` "whole" measures bits against the
    fewest bits of a whole-image candidate (of any candidate if none is
    whole-image), "best" against the fewest bits of any candidate. If no
    candidate passes both bits checks the one with the fewest bits is
    chosen."""
    if reference not in ("whole", "best"):
        raise ValueError(f"reference must be 'whole' or 'best', not {reference!r}")
    cands = [(None if p is None else tuple(p), K) for p in patches for K in interleaves]
    if rows:
        cands.append((None, ROWS))
    table = []
    stream = torch.cuda.current_stream(model.device)
    for patch, K in cands:
        data, offs = model.encode(imgs, order=WAVEFRONT, patch=patch, interleave=K)
        per_img = payload_bits(data, offs)
        bits = sum(per_img)
        cost = max((image_streams(int(t.shape[0]), int(t.shape[1]), patch, K) * STREAM_BITS / max(b, 1)
                    for t, b in zip(imgs, per_img)), default=0.0)
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
        table.append({"patch": patch, "interleave": K, "decode_ms": statistics.median(times), "bits": bits,
                      "stream_cost": cost})
        del ws
    whole = [r["bits"] for r in table if r["patch"] is None]
    ref = min(whole) if reference == "whole" and whole else min(r["bits"] for r in table)
    for r in table:
        r["ok"] = r["bits"] <= ref * (1.0 + max_bits_cost) and r["stream_cost"] <= max_bits_cost
    ok = [r for r in table if r["ok"]]
    choice = min(ok, key=lambda r: r["decode_ms"]) if ok else min(table, key=lambda r: r["bits"])
    return choice, table
