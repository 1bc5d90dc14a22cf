"""Decode-time sweeps over model size and image size on one GPU: the serial
raster decoder against the wavefront decoder (Sec. 3, Algorithm 1), whole
image and with patches, in the manner of the paper's Table 2 (decode time
per image for 0/1/3 residual blocks at 32x32, and for image sides 32 to
1024 with no block). Inputs are the seeded smooth synthetic images of the
shared input recipe; models are its random-init local models with h = 3.
Whole images decode with one stream per lane (one wave per image) and with
one stream per image row (the rows of a wavefront step decoded together, in
pipelined bands of rows).

    python -m paper_2201_05213_amd.sweep > table.md
    python -m paper_2201_05213_amd.sweep --patches   # large batch: patch shape x streams
    python -m paper_2201_05213_amd.sweep --patches --shapes 84x64,86x64 --streams 4
"""
from __future__ import annotations

import argparse
import sys

import numpy as np
import torch

import paper_2201_05213_amd as nx
import synth

__all__ = ["time_decode", "run"]


def _images(n, H, W, seed):
    """Seeded smooth fields from the shared input recipe: up to 256 pixels a
    side the small-image generator (Gaussian blur sigma 2, 3 step edges), above
    it the large-image one (sigma 4, 20 edges, +-3 uniform noise)."""
    sigma, edges, noise = (2.0, 3, 0) if max(H, W) <= 256 else (4.0, 20, 3)
    return [synth.smooth_field_image(sigma, edges, noise, H, W, seed + k) for k in range(n)]


def time_decode(m, imgs, order, patch=None, interleave=1, reps=3):
    """Median decode time (s) of the batch `imgs` (CUDA uint8 tensors),
    decoding checked exact."""
    data, offs = m.encode(imgs, order=order, patch=patch, interleave=interleave)
    out = [torch.empty_like(t) for t in imgs]
    plan, ws = m.decode_prepare(out, order=order, patch=patch, interleave=interleave)
    status = torch.empty(len(imgs), dtype=torch.int32, device=m.device)
    m.decode_run(plan, data, offs, status, ws)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(out, imgs)), "decode mismatch"
    times = []
    stream = torch.cuda.current_stream(m.device)
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        m.decode_run(plan, data, offs, status, ws)
        b.record(stream)
        b.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    return float(np.median(times))


def _model(h, C, nb, seed):
    """Random-init local model from the shared weight recipe
    (U(+-1/sqrt(fan_in)) for every weight and bias)."""
    return nx.Model(synth.write_blob(h, C, nb, synth.init_params(h, C, nb, seed)))


def run(C: int = 32, raster_rows: int = 8, out=sys.stdout):
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pr = lambda s: print(s, file=out, flush=True)  # noqa: E731
    pr(f"### Model size (h = 3, C = {C}), one 32x32 image, decode time per image")
    pr("")
    pr("| residual blocks | raster | wavefront | speedup |")
    pr("|---|---|---|---|")
    img32 = [torch.from_numpy(i).to(dev) for i in _images(1, 32, 32, 7)]
    for nb in (0, 1, 3):
        m = _model(3, C, nb, 100 + nb)
        tr = time_decode(m, img32, nx.RASTER)
        tw = time_decode(m, img32, nx.WAVEFRONT)
        pr(f"| {nb} | {tr * 1e3:.2f} ms | {tw * 1e3:.2f} ms | {tr / tw:.1f}x |")
    pr("")
    pr(f"### Image size (h = 3, C = {C}, no block), decode time per image")
    pr("")
    pr("| side | raster | wavefront, whole image | speedup | whole image, row streams | speedup "
       "| wavefront + 64x64 patches, 4 streams | speedup |")
    pr("|---|---|---|---|---|---|---|---|")
    m = _model(3, C, 0, 100)
    for side in (32, 64, 128, 1024):
        img = [torch.from_numpy(i).to(dev) for i in _images(1, side, side, 11 + side)]
        if side <= 128:
            tr = time_decode(m, img, nx.RASTER)
            rnote = ""
        else:
            # raster time is the same per pixel on every row: a strip of rows, scaled
            strip = [img[0][:raster_rows].contiguous()]
            tr = time_decode(m, strip, nx.RASTER, reps=1) * side / raster_rows
            rnote = f" ({raster_rows}-row strip, scaled)"
        tw = time_decode(m, img, nx.WAVEFRONT, reps=2 if side > 128 else 3)
        trw = time_decode(m, img, nx.WAVEFRONT, interleave=nx.ROWS)
        tp = time_decode(m, img, nx.WAVEFRONT, patch=(64, 64), interleave=4) if side >= 64 else float("nan")
        sp = f"{tp * 1e3:.2f} ms | {tr / tp:.0f}x" if side >= 64 else "n/a | n/a"
        pr(f"| {side} | {tr * 1e3:.2f} ms{rnote} | {tw * 1e3:.2f} ms | {tr / tw:.1f}x | {trw * 1e3:.2f} ms | "
           f"{tr / trw:.0f}x | {sp} |")


def run_patches(out=sys.stdout, shapes=((32, 64), (64, 64), (80, 64), (96, 64), (112, 64), (128, 64), (64, 96),
                                       (64, 128), (96, 96), (128, 128)),
                streams=(16, 8, 4), reps=3):
    """Decode time of the large batch (4 x 1024^2 + 2 x 2048x1536, model B,
    wavefront order) by patch shape and rANS streams per lane."""
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    pr = lambda s: print(s, file=out, flush=True)  # noqa: E731
    ts = [torch.from_numpy(i).to(dev) for i in synth.workload_images("large6")]
    m = nx.Model(synth.model_blob("B")[0])
    pr("| patch (rows x cols) | lanes | waves/CU | " + " | ".join(f"{k} stream(s)" for k in streams) + " |")
    pr("|---|---|---|" + "---|" * len(streams))
    for patch in shapes:
        cells, lanes, waves = [], 0, 0
        for K in streams:
            data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=K)
            outs = [torch.empty_like(t) for t in ts]
            plan, ws = m.decode_prepare(outs, order=nx.WAVEFRONT, patch=patch, interleave=K)
            lanes, waves = plan.n_lanes, plan.waves
            cells.append(f"{time_decode(m, ts, nx.WAVEFRONT, patch=patch, interleave=K, reps=reps) * 1e3:.2f} ms")
            del ws
        pr(f"| {patch[0]} x {patch[1]} | {lanes} | {waves} | " + " | ".join(cells) + " |")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--channels", type=int, default=32)
    ap.add_argument("--raster-rows", type=int, default=8)
    ap.add_argument("--patches", action="store_true",
                    help="instead: decode time of the large batch by patch shape and streams per lane")
    ap.add_argument("--shapes", default=None,
                    help="with --patches: comma-separated ROWSxCOLS patch shapes (default: a fixed set)")
    ap.add_argument("--streams", default="16,8,4", help="with --patches: comma-separated streams per lane")
    a = ap.parse_args()
    if a.patches:
        kw = {"streams": tuple(int(k) for k in a.streams.split(","))}
        if a.shapes:
            kw["shapes"] = tuple(tuple(int(v) for v in sh.split("x")) for sh in a.shapes.split(","))
        run_patches(**kw)
    else:
        run(a.channels, a.raster_rows)
