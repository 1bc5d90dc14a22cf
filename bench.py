"""Benchmark: decoded pixels/s on one MI355X, wavefront + patch decode vs the
same GPU's raster decode, bits/dim gap vs the FP64 oracle.

Workload (synthetic, seeded): 4 images of 1024x1024 and 2 of 2048x1536 uint8
RGB (smooth random fields, sigma 4 px, 20 step edges, +-3 integer noise),
coded with the h=3, 64-channel, 2-block local model (random-init weights) in
the wavefront order with independent patches of 64 columns, each patch one
lane of 16 interleaved rANS streams (one per row of a 16-row group); the
patch height is the shortest that keeps the batch at two lanes per SIMD (86
rows on 256 CUs: 1,920 lanes). One timed step = one decode
of the whole batch from containers already resident in HBM, by default in the
sheared layout (ShearLoC, Sec. 3.1 and Algorithm 2); the unsheared wavefront
decoder (Algorithm 1) is timed on the same containers as a second leg.

Prints one JSON line (see the keys below); --gpus N > 1 is refused: this
path runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32 = 157.3e12  # MI355X dense FP32 (matrix) FLOP/s
CALIB_BYTES = 256 << 20  # copy kernel used to calibrate the HBM byte counters

# HBM bytes per decoder launch on this workload from two counter passes
# (FETCH_SIZE, WRITE_SIZE), each scaled by the same counter's reading for a
# 256 MiB device copy, per decoder layout; valid only for the kernel sources,
# patch shape and streams per lane they were taken on
DECODE_TRAFFIC = {
    "sheared": {"src_sha": "fd38217a5f6439eb", "patch": (82, 64), "interleave": 16,
                "fetch_kib": 38035.7, "write_kib": 748684.8, "fetch_scale": 1.99982, "write_scale": 1.0},
}
KERNEL_SOURCES = ("nx_kernels.hip", "nx_device.hpp", "nx_layout.hpp", "nx_kernels.hpp", "nx_order.hpp")


def kernel_sources_sha() -> str:
    """sha256[:16] of the coder's kernel sources and of the compiler flags
    they are built with."""
    import hashlib

    from paper_2201_05213_amd import build as nxbuild

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2201_05213_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    h.update(repr(nxbuild.coder_flags()).encode())
    return h.hexdigest()[:16]


def decode_traffic_bytes(layout: str, patch, interleave: int):
    t = DECODE_TRAFFIC.get(layout)
    if t is None or kernel_sources_sha() != t["src_sha"] or tuple(patch) != t["patch"] or interleave != t["interleave"]:
        return None
    return round(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]))


def macs_per_px(h: int, C: int, nb: int) -> int:
    """Multiply-accumulates of the local model per pixel: causal taps of the
    first layer, the 1x1 blocks and the 100-output head."""
    return 2 * h * (h + 1) * 3 * C + nb * 2 * C * C + 100 * C


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- oracle pool
# The CPU baseline runs the oracle (FP64 C, one lane per call) in worker
# processes, one per core of the box's share; each worker loads the model once.
_ORACLE = None


def _oracle_init(blob: bytes) -> None:
    global _ORACLE
    sys.path.insert(0, ROOT)
    import oracle

    _ORACLE = oracle.Model.from_blob(blob)


def _oracle_job(job):
    """('enc', lane) -> container; ('dec', lane, container) -> None (checked
    exact); ('stats', lane) -> quantised ideal bits."""
    import numpy as np

    kind, lane = job[0], job[1]
    if kind == "enc":
        return _ORACLE.encode(lane, 1)
    if kind == "dec":
        out = _ORACLE.decode(job[2], lane.shape[0], lane.shape[1], 1)
        assert np.array_equal(out, lane), "oracle round trip failed"
        return None
    return _ORACLE.stats(lane)["qbits"]


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cpus() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--patch", default="auto",
                    help="patch shape ROWSxCOLS, one number for square patches, or auto: the shortest 64-column "
                         "patch that keeps the batch at two lanes per SIMD (tune.balanced_patch)")
    ap.add_argument("--interleave", type=int, default=16, help="rANS streams per lane (1, 2, 4, 8 or 16)")
    ap.add_argument("--layout", choices=("sheared", "unsheared"), default="sheared",
                    help="decoder layout of the headline decode: sheared (ShearLoC, Algorithm 2) or the "
                         "unsheared wavefront decoder (Algorithm 1); the other is timed as a second leg")
    ap.add_argument("--raster-rows", type=int, default=32,
                    help="rows of the 1024-wide strip the raster baseline decodes")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-lanes", type=int, default=32, help="lanes of image 0 the oracle decodes on one thread")
    ap.add_argument("--cpu-procs", type=int, default=16,
                    help="oracle processes of the all-cores leg (at most the CPUs this process may use)")
    ap.add_argument("--train-steps", type=int, default=50,
                    help="timed training steps (model B, 64 random 32x32 crops, Adam); 0 skips the leg")
    ap.add_argument("--no-trained", action="store_true",
                    help="skip the trained-model leg (model B after the 2000-step training recipe, trained on the "
                         "CPU by the oracle: decode time and the bits gap at about 4 bits/dim)")
    ap.add_argument("--profile-rows", action="store_true",
                    help="only decode image 0 (1024^2) as a whole-image lane with row streams, warmup + steps "
                         "times (for profiler runs of the row-stream decoder; prints no JSON)")
    ap.add_argument("--profile-train", action="store_true",
                    help="only run warmup + steps training steps of the training leg (model B, 64 random 32x32 "
                         "crops, forward + backward + Adam; for profiler runs of the training kernels; prints no "
                         "JSON)")
    ap.add_argument("--profile", action="store_true",
                    help="time only the batch decode, then run the full-image pass and the encode three times "
                         "each and a known-size copy for counter calibration (for profiler runs; prints no "
                         "JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the library has no multi-GPU path"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2201_05213_amd as nx
    import synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.profile_train:
        from paper_2201_05213_amd import blob as nxblob, train as nxtrain

        tdims, tparams = nxblob.params_from_blob(synth.model_blob("B")[0])
        pool = torch.from_numpy(synth.training_pool(n=512)).to(dev)
        rng = np.random.Generator(np.random.PCG64(5_999_999))
        p = torch.nn.Parameter(torch.from_numpy(tparams).to(dev))
        opt = torch.optim.Adam([p], lr=1e-3, fused=True)
        batches = [nxtrain.random_crops(pool, 64, 32, rng) for _ in range(args.warmup + args.steps)]
        torch.cuda.synchronize()
        for x in batches:
            opt.zero_grad(set_to_none=True)
            (nxtrain.nll_bits(p, tdims, x).sum() / x.numel()).backward()
            opt.step()
        torch.cuda.synchronize()
        log(f"[bench] profile-train mode: {args.warmup + args.steps} training steps done")
        return
    t0 = time.time()
    imgs = synth.workload_images("large6")
    log(f"[bench] generated {len(imgs)} images in {time.time() - t0:.1f}s")
    blob, dims = synth.model_blob("B")
    m = nx.Model(blob)
    ts = [torch.from_numpy(i).to(dev) for i in imgs]
    shapes = [i.shape[:2] for i in imgs]
    npx = sum(h * w for h, w in shapes)
    if args.patch == "auto":
        from paper_2201_05213_amd import tune as nxtune

        ph, pw = nxtune.balanced_patch(shapes)
    else:
        ph, pw = (int(v) for v in (args.patch.split("x") if "x" in args.patch else (args.patch, args.patch)))
    patch = (ph, pw)
    pname = f"{ph}x{pw}"
    if args.profile_rows:
        d0, o0 = m.encode([ts[0]], order=nx.WAVEFRONT, interleave=nx.ROWS)
        out0 = [torch.empty_like(ts[0])]
        plan0, ws0 = m.decode_prepare(out0, order=nx.WAVEFRONT, interleave=nx.ROWS)
        st0 = torch.empty(1, dtype=torch.int32, device=dev)
        for _ in range(args.warmup + args.steps):
            m.decode_run(plan0, d0, o0, st0, ws0)
        torch.cuda.synchronize()
        assert int(st0[0]) == 0 and torch.equal(out0[0], ts[0])
        log(f"[bench] profile-rows mode: {args.warmup + args.steps} decodes of one 1024^2 image done")
        return
    lanes_x = -(-1024 // pw)  # lanes across a 1024-wide image

    def lane_crop(img, q):
        ly, lx = divmod(q, lanes_x)
        return np.ascontiguousarray(img[ly * ph:(ly + 1) * ph, lx * pw:(lx + 1) * pw])

    # encode once (untimed), containers stay in HBM
    torch.cuda.synchronize()
    e0 = time.time()
    data, offs = m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave)
    torch.cuda.synchronize()
    enc_s = time.time() - e0
    log(f"[bench] encoded {npx} px in {enc_s:.3f}s, {data.numel()} bytes")

    outs = [torch.empty_like(t) for t in ts]
    L = nx.load()
    import ctypes
    dec_order = nx.SHEARED if args.layout == "sheared" else nx.WAVEFRONT
    alt_order = nx.WAVEFRONT if args.layout == "sheared" else nx.SHEARED
    o = nx._opts(dec_order, patch, args.interleave)
    arr = nx._images(outs)
    ws = m.workspace(arr, len(outs), o)
    status = torch.empty(len(outs), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream(dev)

    def decode_once():
        rc = L.nellox_decode(m._h, len(outs), data.data_ptr(), offs.data_ptr(), ctypes.byref(o), arr,
                             status.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"nellox_decode returned {rc}")

    for _ in range(args.warmup):
        decode_once()
    torch.cuda.synchronize()
    log("[bench] warmup done")

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    w0 = time.time()
    for s, e in evs:
        s.record(stream)
        decode_once()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.time() - w0
    # every timed step rewrote the same outputs: check the last one
    assert all(torch.equal(a, b) for a, b in zip(outs, ts)), "round trip failed"
    assert int(status.abs().sum()) == 0
    log("[bench] round trip exact")
    times = [s.elapsed_time(e) / 1e3 for s, e in evs]
    step_s = sum(times) / len(times)
    value = npx / step_s
    log(f"[bench] decode step {step_s * 1e3:.2f} ms (wall {wall / args.steps * 1e3:.2f} ms/step), "
        f"{value / 1e6:.1f} Mpx/s")

    flops_per_px = 2 * macs_per_px(dims["h"], dims["C"], dims["n_blocks"])
    achieved = flops_per_px * npx / step_s

    if args.profile:
        # the full-image pass alone (the fused per-pixel routine, through the
        # symbol hook with no sum) and whole encodes, three times each, warm
        pws = m.workspace(arr, len(ts), o)
        psym = torch.empty(npx * 3, dtype=torch.int32, device=dev)
        parr = nx._images(ts)
        po = nx._opts(nx.WAVEFRONT, patch)
        for _ in range(3):
            rc = L.nellox_debug_symbols(m._h, len(ts), parr, ctypes.byref(po), psym.data_ptr(), None,
                                        pws.data_ptr(), pws.numel(), ctypes.c_void_p(stream.cuda_stream))
            if rc != 0:
                raise RuntimeError(f"nellox_debug_symbols returned {rc}")
        for _ in range(3):
            m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave, ws=pws, sync=False)
        torch.cuda.synchronize()
        del pws, psym
        # a plain device copy of known size: its FETCH_SIZE / WRITE_SIZE
        # counters scale the decoder's into bytes
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] profile mode: {CALIB_BYTES} B copy x3 done")
        return

    # encoder: the whole nellox_encode (full-image pass, per-stream rANS,
    # container assembly), and the full-image pass alone (the fused per-pixel
    # routine: gather, network, mixture, two CDF points per channel), timed
    # through the symbol hook that runs just that pass
    enc_ws = m.workspace(arr, len(ts), o)
    for _ in range(2):
        m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave, ws=enc_ws, sync=False)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    nrep = max(3, args.steps // 2)
    ev[0].record(stream)
    for _ in range(nrep):
        m.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave, ws=enc_ws, sync=False)
    ev[1].record(stream)
    sym_buf = torch.empty(npx * 3, dtype=torch.int32, device=dev)
    in_arr = nx._images(ts)
    o1 = nx._opts(nx.WAVEFRONT, patch)
    for _ in range(nrep):
        rc = L.nellox_debug_symbols(m._h, len(ts), in_arr, ctypes.byref(o1), sym_buf.data_ptr(), None,
                                    enc_ws.data_ptr(), enc_ws.numel(), ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"nellox_debug_symbols returned {rc}")
    ev[2].record(stream)
    torch.cuda.synchronize()
    enc_step = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
    pass_step = ev[1].elapsed_time(ev[2]) / 1e3 / nrep
    enc_rec = {"px_per_s": npx / enc_step, "ms": enc_step * 1e3, "pass_ms": pass_step * 1e3,
               "pass_tflops": flops_per_px * npx / pass_step / 1e12,
               "pass_frac_fp32_peak": flops_per_px * npx / pass_step / PEAK_FP32}
    log(f"[bench] encode {enc_step * 1e3:.2f} ms ({npx / enc_step / 1e6:.0f} Mpx/s); full-image pass "
        f"{pass_step * 1e3:.2f} ms, {enc_rec['pass_tflops']:.1f} TFLOP/s ({enc_rec['pass_frac_fp32_peak'] * 100:.1f}% "
        f"of FP32 peak)")

    # the same containers decoded in the other layout
    plan2, ws2 = m.decode_prepare(outs, order=alt_order, patch=patch, interleave=args.interleave)
    for _ in range(2):
        m.decode_run(plan2, data, offs, status, ws2)
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(nrep):
        m.decode_run(plan2, data, offs, status, ws2)
    ev[1].record(stream)
    torch.cuda.synchronize()
    assert all(torch.equal(a, b) for a, b in zip(outs, ts)), "round trip failed (other layout)"
    assert int(status.abs().sum()) == 0
    alt_step = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
    alt_name = "unsheared" if args.layout == "sheared" else "sheared"
    alt_rec = {"layout": alt_name, "px_per_s": npx / alt_step, "ms": alt_step * 1e3,
               "headline_speedup": alt_step / step_s,
               "traffic": decode_traffic_bytes(alt_name, patch, args.interleave),
               "sample": f"the timed containers decoded in the {alt_name} layout (prepared run), round trip checked"}
    log(f"[bench] {alt_name} decode {alt_step * 1e3:.2f} ms ({npx / alt_step / 1e6:.0f} Mpx/s); the {args.layout} "
        f"headline is {alt_step / step_s:.3f}x faster")
    del ws2

    # variants of the large-image workload, in the headline's decoder layout:
    # model B on 64x64 and 32x32 patches, and the h = 2, 32-channel model C on
    # the headline's patches and on 64x64 (prepared runs, round trips checked)
    variants = {}
    mc = nx.Model(synth.model_blob("C")[0])
    for mname, vpatch in dict.fromkeys((("B", (64, 64)), ("B", (32, 32)), ("C", patch), ("C", (64, 64)))):
        if mname == "B" and vpatch == patch:
            continue  # the headline itself
        vname = f"model_{mname}_p{vpatch[0]}x{vpatch[1]}"
        mv = m if mname == "B" else mc
        vd, vo = mv.encode(ts, order=nx.WAVEFRONT, patch=vpatch, interleave=args.interleave)
        vplan, vws = mv.decode_prepare(outs, order=dec_order, patch=vpatch, interleave=args.interleave)
        mv.decode_run(vplan, vd, vo, status, vws)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(nrep):
            mv.decode_run(vplan, vd, vo, status, vws)
        ev[1].record(stream)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ts)), f"round trip failed ({vname})"
        assert int(status.abs().sum()) == 0
        vstep = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
        vh, vC, vnb = (synth.MODEL_DIMS[mname][k] for k in ("h", "C", "n_blocks"))
        vflops = 2 * macs_per_px(vh, vC, vnb) * npx / vstep
        variants[vname] = {"ms": vstep * 1e3, "px_per_s": npx / vstep, "tflops": vflops / 1e12,
                           "frac_fp32_peak": vflops / PEAK_FP32, "patch": list(vpatch), "layout": args.layout,
                           "model": f"h={vh}, C={vC}, {vnb} block(s)"}
        log(f"[bench] {vname}: decode {vstep * 1e3:.2f} ms ({npx / vstep / 1e6:.0f} Mpx/s, "
            f"{100 * vflops / PEAK_FP32:.1f}% of FP32 peak)")
        del vws

    # the other batch workloads with model B: 512 images of 32x32 (one lane
    # per image, the streams chosen by the autotuner) and the uneven 64-image
    # batch with the patch shape and streams chosen by the autotuner (the
    # fastest layout within 0.1% of whole-image coding's bits whose streams
    # cost under 0.1%)
    from paper_2201_05213_amd import tune

    def time_workload(wimgs, wpatch, K):
        wd, wo = m.encode(wimgs, order=nx.WAVEFRONT, patch=wpatch, interleave=K)
        wout = [torch.empty_like(t) for t in wimgs]
        wst = torch.empty(len(wimgs), dtype=torch.int32, device=dev)
        wplan, wws = m.decode_prepare(wout, order=nx.WAVEFRONT, patch=wpatch, interleave=K)
        m.decode_run(wplan, wd, wo, wst, wws)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(nrep):
            m.decode_run(wplan, wd, wo, wst, wws)
        ev[1].record(stream)
        for _ in range(nrep):
            m.encode(wimgs, order=nx.WAVEFRONT, patch=wpatch, interleave=K, sync=False)
        ev[2].record(stream)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(wout, wimgs)) and int(wst.abs().sum()) == 0
        wpx = sum(int(t.shape[0]) * int(t.shape[1]) for t in wimgs)
        dms = ev[0].elapsed_time(ev[1]) / nrep
        ems = ev[1].elapsed_time(ev[2]) / nrep
        return {"images": len(wimgs), "pixels": wpx, "patch": None if wpatch is None else list(wpatch),
                "interleave": K, "decode_ms": dms, "decode_px_per_s": wpx / dms * 1e3, "encode_ms": ems,
                "encode_px_per_s": wpx / ems * 1e3}

    workloads = {}
    b512 = [torch.from_numpy(i).to(dev) for i in synth.workload_images("batch512x32")]
    # one lane per image (the workload's own layout); the tuner picks its streams
    bchoice, btab = tune.autotune(m, b512, patches=(None,), rows=False)
    workloads["batch512x32"] = time_workload(b512, None, bchoice["interleave"])
    workloads["batch512x32"]["autotuned"] = True
    workloads["batch512x32"]["autotune_table"] = [
        {"interleave": r["interleave"], "decode_ms": r["decode_ms"], "bits": r["bits"], "stream_cost": r["stream_cost"],
         "ok": r["ok"]} for r in btab]
    un64 = [torch.from_numpy(i).to(dev) for i in synth.workload_images("uneven64")]
    choice, utab = tune.autotune(m, un64)
    workloads["uneven64"] = time_workload(un64, choice["patch"], choice["interleave"])
    workloads["uneven64"]["autotuned"] = True
    workloads["uneven64"]["autotune_table"] = [
        {"patch": None if r["patch"] is None else list(r["patch"]), "interleave": r["interleave"],
         "decode_ms": r["decode_ms"], "bits": r["bits"], "stream_cost": r["stream_cost"], "ok": r["ok"]}
        for r in utab]
    del b512, un64
    for wn, w in workloads.items():
        log(f"[bench] {wn}: decode {w['decode_ms']:.2f} ms ({w['decode_px_per_s'] / 1e6:.0f} Mpx/s), encode "
            f"{w['encode_ms']:.2f} ms, patch {w['patch']}, {w['interleave']} stream(s)")

    # ancestral sampling of the same batch shape with the decoder's schedule
    # (each symbol the inverse quantised CDF at a Philox slot; no coder)
    smp_out = [torch.empty_like(t) for t in ts]
    smp_arr = nx._images(smp_out)
    seeds = (ctypes.c_uint64 * len(ts))(*[1000 + k for k in range(len(ts))])

    def sample_once():
        rc = L.nellox_sample(m._h, len(ts), seeds, ctypes.byref(o1), smp_arr, enc_ws.data_ptr(), enc_ws.numel(),
                             ctypes.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise RuntimeError(f"nellox_sample returned {rc}")

    for _ in range(2):
        sample_once()
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(nrep):
        sample_once()
    ev[1].record(stream)
    torch.cuda.synchronize()
    smp_step = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
    smp_rec = {"px_per_s": npx / smp_step, "ms": smp_step * 1e3,
               "tflops": flops_per_px * npx / smp_step / 1e12,
               "frac_fp32_peak": flops_per_px * npx / smp_step / PEAK_FP32,
               "sample": "the decode batch's shapes, wavefront order, same patches; one seed per image"}
    log(f"[bench] sampling {smp_step * 1e3:.2f} ms ({npx / smp_step / 1e6:.0f} Mpx/s, "
        f"{smp_rec['frac_fp32_peak'] * 100:.1f}% of FP32 peak)")

    # one 1024x1024 image alone: wavefront+patch latency
    one = [ts[0]]
    d1, o1 = m.encode(one, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave)
    for _ in range(2):
        m.decode(d1, o1, [shapes[0]], order=nx.WAVEFRONT, patch=patch, interleave=args.interleave)
    torch.cuda.synchronize()
    s1, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s1.record(stream)
    m.decode(d1, o1, [shapes[0]], order=nx.WAVEFRONT, patch=patch, sync=False, interleave=args.interleave)
    e1.record(stream)
    torch.cuda.synchronize()
    one_s = s1.elapsed_time(e1) / 1e3
    log(f"[bench] one 1024^2 image, wavefront+patch: {one_s * 1e3:.2f} ms")

    # raster baseline on the same GPU: a 1024-wide strip decoded pixel by
    # pixel in one lane; raster cost per pixel does not depend on the row, so
    # the full-image time is the strip time scaled by 1024 / rows
    rows = args.raster_rows
    strip = ts[0][:rows].contiguous()
    d2, o2 = m.encode([strip], order=nx.RASTER)
    m.decode(d2, o2, [(rows, 1024)], order=nx.RASTER)
    torch.cuda.synchronize()
    s2, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s2.record(stream)
    (rout,), _ = m.decode(d2, o2, [(rows, 1024)], order=nx.RASTER, sync=False)
    e2.record(stream)
    torch.cuda.synchronize()
    assert torch.equal(rout, strip)
    strip_s = s2.elapsed_time(e2) / 1e3
    raster_pxs = rows * 1024 / strip_s
    raster_full_s = strip_s * 1024 / rows
    log(f"[bench] raster: {rows}x1024 strip {strip_s:.3f}s -> {raster_pxs:.0f} px/s, "
        f"1024^2 extrapolated {raster_full_s:.1f}s")

    # the paper's exact method: whole-image lanes (no patch borders), one rANS
    # stream per image row, every row of a wavefront step at once, bands of 16
    # rows pipelined across CUs; one 1024^2 image alone (latency, against the
    # raster decode) and the whole batch (throughput, bits/dim against the
    # oracle's whole-image ideal when tests/golden/patch_cost.json holds it)
    whole_rec = {}
    for wname, wm in (("B", m), ("B_trained", None)):
        if wm is None:
            tpath = os.path.join(ROOT, "tests", "golden", "model_b_trained.nlxw")
            if not os.path.exists(tpath):
                continue
            with open(tpath, "rb") as f:
                wm = nx.Model(f.read())
        rd, ro = wm.encode(ts, order=nx.WAVEFRONT, interleave=nx.ROWS)
        rplan, rws = wm.decode_prepare(outs, order=nx.WAVEFRONT, interleave=nx.ROWS)
        wm.decode_run(rplan, rd, ro, status, rws)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(3):
            wm.decode_run(rplan, rd, ro, status, rws)
        ev[1].record(stream)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ts)) and int(status.abs().sum()) == 0
        batch_ms = ev[0].elapsed_time(ev[1]) / 3
        rbits = float(sum(nx.payload_bits(rd, ro)))
        # one 1024^2 image alone
        r1d, r1o = wm.encode([ts[0]], order=nx.WAVEFRONT, interleave=nx.ROWS)
        p1, w1 = wm.decode_prepare([outs[0]], order=nx.WAVEFRONT, interleave=nx.ROWS)
        st1 = status[:1]
        wm.decode_run(p1, r1d, r1o, st1, w1)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(3):
            wm.decode_run(p1, r1d, r1o, st1, w1)
        ev[1].record(stream)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], ts[0]) and int(st1.abs().sum()) == 0
        one_ms = ev[0].elapsed_time(ev[1]) / 3
        rec = {"one_1024_ms": one_ms, "speedup_vs_raster_1024": None, "batch_ms": batch_ms,
               "batch_px_per_s": npx / batch_ms * 1e3, "bits_per_dim": rbits / (3 * npx),
               "bands": int(rplan.n_bands)}
        opath = os.path.join(ROOT, "tests", "golden", "patch_cost.json")
        if os.path.exists(opath):
            with open(opath) as f:
                ores = json.load(f)["results"]
            if wname in ores:
                ideal = ores[wname]["large6"]["whole"]["qbits"]
                rec["gap_vs_oracle_whole_image_ideal"] = (rbits - ideal) / ideal
        whole_rec[wname] = rec
        del rws, w1
        log(f"[bench] whole-image lanes, row streams, model {wname}: one 1024^2 image {one_ms:.1f} ms; batch "
            f"{batch_ms:.1f} ms ({npx / batch_ms / 1e3:.0f} Mpx/s, {rplan.n_bands} bands); "
            f"{rbits / (3 * npx):.4f} bits/dim" + (f", gap {100 * rec['gap_vs_oracle_whole_image_ideal']:.4f}% vs "
            f"the oracle's whole-image ideal" if "gap_vs_oracle_whole_image_ideal" in rec else ""))

    # bits/dim: coded lane payloads vs the oracle's quantised ideal on sampled lanes
    cont = data.cpu().numpy()
    offs_h = offs.cpu().numpy()
    total_payload_bits = 0
    for k in range(len(imgs)):
        c = cont[offs_h[k]:offs_h[k + 1]]
        nl = int.from_bytes(bytes(c[28:32]), "little")
        total_payload_bits += 8 * (len(c) - 32 - 4 * nl * int(c[7]))
    bpd = total_payload_bits / (3 * npx)
    gap = None
    cpu = None
    if not args.no_cpu:
        import multiprocessing as mp

        import oracle

        c0 = cont[offs_h[0]:offs_h[1]]
        nl0 = int.from_bytes(bytes(c0[28:32]), "little")
        K0 = int(c0[7])
        ends = np.frombuffer(bytes(c0[32:32 + 4 * nl0 * K0]), dtype="<u4").astype(np.int64)
        # bits per lane: the sum of its K stream payloads
        lane_bits = np.diff(np.concatenate([[0], ends])).reshape(nl0, K0).sum(axis=1) * 8
        crops = [lane_crop(imgs[0], q) for q in range(nl0)]
        procs = max(1, min(args.cpu_procs, usable_cpus()))
        with mp.get_context("spawn").Pool(procs, initializer=_oracle_init, initargs=(blob,)) as pool:
            pool.map(_oracle_job, [("stats", crops[0][:4, :4].copy())] * procs)  # workers up and loaded
            t0 = time.time()
            encs = pool.map(_oracle_job, [("enc", c) for c in crops], chunksize=1)
            cpu_enc_s = time.time() - t0
            t0 = time.time()
            pool.map(_oracle_job, [("dec", c, e) for c, e in zip(crops, encs)], chunksize=1)
            cpu_dec_s = time.time() - t0
            ideals = pool.map(_oracle_job, [("stats", c) for c in crops], chunksize=1)
        # the gap over every lane of image 0
        ideal, got = float(sum(ideals)), float(lane_bits.sum())
        gap = (got - ideal) / ideal
        log(f"[bench] gap on all {nl0} lanes of image 0: {gap * 100:.4f}% ({got:.0f} vs {ideal:.1f} bits, "
            f"{(got - ideal) / (nl0 * K0):.1f} bits per stream)")
        # one thread: the oracle in this process on the first lanes
        om = oracle.Model.from_blob(blob)
        c1 = time.time()
        for c, enc in zip(crops[:args.cpu_lanes], encs):
            dec = om.decode(enc, c.shape[0], c.shape[1], 1)
            assert np.array_equal(dec, c)
        cpu1_s = time.time() - c1
        lpx = sum(c.shape[0] * c.shape[1] for c in crops)
        one_px = sum(c.shape[0] * c.shape[1] for c in crops[:args.cpu_lanes])
        cpu = {"value": lpx / cpu_dec_s, "unit": "decoded px/s", "cores": procs, "kind": "oracle",
               "encode_px_per_s": lpx / cpu_enc_s, "decode_px_per_s_1thread": one_px / cpu1_s,
               "nproc": os.cpu_count(), "usable_cpus": usable_cpus(), "cpu_model": cpu_model(),
               "sample": f"all {nl0} {pname} lanes of image 0 (1024x1024, {lpx} px), wavefront order, FP64 C "
                         f"oracle, one lane per call in {procs} processes: encode {cpu_enc_s:.1f} s, decode "
                         f"{cpu_dec_s:.1f} s; one thread: {args.cpu_lanes} lanes decoded in {cpu1_s:.1f} s"}
        log(f"[bench] oracle CPU ({procs} processes, {cpu['cpu_model']}): decode {cpu['value']:.0f} px/s, encode "
            f"{cpu['encode_px_per_s']:.0f} px/s; one thread decode {cpu['decode_px_per_s_1thread']:.0f} px/s")

    # training leg: one step = forward + hand-written backward + Adam on
    # 64 random 32x32 crops, model B
    train_rec = None
    if args.train_steps > 0:
        from paper_2201_05213_amd import blob as nxblob, train as nxtrain

        tdims, tparams = nxblob.params_from_blob(blob)
        pool = torch.from_numpy(synth.training_pool(n=512)).to(dev)
        rng = np.random.Generator(np.random.PCG64(5_999_999))
        p = torch.nn.Parameter(torch.from_numpy(tparams).to(dev))
        opt = torch.optim.Adam([p], lr=1e-3, fused=True)
        batches = [nxtrain.random_crops(pool, 64, 32, rng) for _ in range(args.train_steps + 5)]

        def train_step(x):
            opt.zero_grad(set_to_none=True)
            loss = nxtrain.nll_bits(p, tdims, x).sum() / x.numel()
            loss.backward()
            opt.step()

        for x in batches[:5]:
            train_step(x)
        torch.cuda.synchronize()
        ts0, ts1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts0.record(stream)
        for x in batches[5:]:
            train_step(x)
        ts1.record(stream)
        torch.cuda.synchronize()
        tstep = ts0.elapsed_time(ts1) / 1e3 / args.train_steps
        tpx = 64 * 32 * 32
        # forward 1x, backward ~2x the forward's multiply-accumulates
        tflops = 3 * flops_per_px * tpx / tstep
        train_rec = {"step_ms": tstep * 1e3, "px_per_s": tpx / tstep, "tflops_fwd_bwd": tflops / 1e12,
                     "frac_fp32_peak": tflops / PEAK_FP32,
                     "sample": "model B, 64 random 32x32 crops per step, forward + backward + Adam"}
        log(f"[bench] training step {tstep * 1e3:.3f} ms ({tflops / 1e12:.1f} TFLOP/s fwd+bwd)")
        # the same step captured once as a HIP graph (torch.cuda.graph) and
        # replayed on each batch copied into the graph's input buffer: the
        # kernels are those of the eager step, without the host's launch gaps
        try:
            pg = torch.nn.Parameter(torch.from_numpy(tparams).to(dev))
            optg = torch.optim.Adam([pg], lr=1e-3, fused=True, capturable=True)
            sx = batches[0].clone()

            def graph_body():
                loss = nxtrain.nll_bits(pg, tdims, sx).sum() / sx.numel()
                loss.backward()
                optg.step()

            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                for _ in range(3):
                    optg.zero_grad(set_to_none=True)
                    graph_body()
            torch.cuda.current_stream().wait_stream(side)
            optg.zero_grad(set_to_none=True)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                graph_body()
            for x in batches[:5]:
                sx.copy_(x)
                graph.replay()
            torch.cuda.synchronize()
            gs = torch.cuda.current_stream()
            tg0, tg1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            tg0.record(gs)
            for x in batches[5:]:
                sx.copy_(x)
                graph.replay()
            tg1.record(gs)
            torch.cuda.synchronize()
            tgs = tg0.elapsed_time(tg1) / 1e3 / args.train_steps
            train_rec["step_ms_graph"] = tgs * 1e3
            train_rec["frac_fp32_peak_graph"] = 3 * flops_per_px * tpx / tgs / PEAK_FP32
            log(f"[bench] training step as a replayed graph {tgs * 1e3:.3f} ms "
                f"({3 * flops_per_px * tpx / tgs / 1e12:.1f} TFLOP/s fwd+bwd)")
            del graph
        except RuntimeError as e:
            train_rec["step_ms_graph"] = None
            log(f"[bench] training step graph capture failed: {e}")

    # the same workload coded by the trained model B (the 2000-step training
    # recipe, run on the CPU by the oracle; ~4.4 bits/dim here): decode time
    # and, over every lane of image 0, the gap with the configured streams and
    # with one stream
    trained_rec = None
    if not args.no_trained:
        with open(os.path.join(ROOT, "tests", "golden", "model_b_trained.nlxw"), "rb") as f:
            tblob = f.read()
        mt = nx.Model(tblob)
        td, to = mt.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=args.interleave)
        plan3, ws3 = mt.decode_prepare(outs, order=dec_order, patch=patch, interleave=args.interleave)
        mt.decode_run(plan3, td, to, status, ws3)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(nrep):
            mt.decode_run(plan3, td, to, status, ws3)
        ev[1].record(stream)
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(outs, ts)), "round trip failed (trained model)"
        assert int(status.abs().sum()) == 0
        t_step = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
        tc = td.cpu().numpy()
        toh = to.cpu().numpy()
        tbits = 0
        for k in range(len(imgs)):
            c = tc[toh[k]:toh[k + 1]]
            nl = int.from_bytes(bytes(c[28:32]), "little")
            tbits += 8 * (len(c) - 32 - 4 * nl * int(c[7]))
        trained_rec = {"bits_per_dim": tbits / (3 * npx), "decode_ms": t_step * 1e3, "px_per_s": npx / t_step,
                       "model": "model B after 2000 Adam steps (tests/golden/model_b_trained.nlxw)"}
        log(f"[bench] trained model B: {tbits / (3 * npx):.3f} bits/dim, decode {t_step * 1e3:.2f} ms "
            f"({npx / t_step / 1e6:.0f} Mpx/s)")
        del ws3
        # eight streams per lane: half the stream bits of sixteen
        if args.interleave != 8:
            td8, to8 = mt.encode(ts, order=nx.WAVEFRONT, patch=patch, interleave=8)
            plan8, ws8 = mt.decode_prepare(outs, order=dec_order, patch=patch, interleave=8)
            mt.decode_run(plan8, td8, to8, status, ws8)
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(nrep):
                mt.decode_run(plan8, td8, to8, status, ws8)
            ev[1].record(stream)
            torch.cuda.synchronize()
            assert all(torch.equal(a, b) for a, b in zip(outs, ts)) and int(status.abs().sum()) == 0
            t8 = ev[0].elapsed_time(ev[1]) / 1e3 / nrep
            trained_rec["decode_ms_k8"] = t8 * 1e3
            trained_rec["px_per_s_k8"] = npx / t8
            log(f"[bench] trained model B, 8 streams: decode {t8 * 1e3:.2f} ms ({npx / t8 / 1e6:.0f} Mpx/s)")
            del ws8, td8
        if not args.no_cpu:
            import multiprocessing as mp

            crops = [lane_crop(imgs[0], q) for q in range(lanes_x * -(-1024 // ph))]
            procs = max(1, min(args.cpu_procs, usable_cpus()))
            with mp.get_context("spawn").Pool(procs, initializer=_oracle_init, initargs=(tblob,)) as pool:
                ideal = float(sum(pool.map(_oracle_job, [("stats", c) for c in crops], chunksize=1)))
            for K in sorted({args.interleave, 8, 1}):
                dK, oK = mt.encode([ts[0]], order=nx.WAVEFRONT, patch=patch, interleave=K)
                c0 = dK.cpu().numpy()
                nl0 = int.from_bytes(bytes(c0[28:32]), "little")
                got = 8.0 * (len(c0) - 32 - 4 * nl0 * K)
                trained_rec[f"gap_vs_oracle_ideal_k{K}"] = (got - ideal) / ideal
                log(f"[bench] trained model B, {K} stream(s): gap on all {nl0} lanes of image 0 "
                    f"{100 * (got - ideal) / ideal:.4f}% ({(got - ideal) / (nl0 * K):.1f} bits per stream)")
            trained_rec["gap_sample"] = f"all {len(crops)} {pname} lanes of image 0"

    # what the patches cost in bits: the quantised ideal code length (the
    # encoder's own CDFs, every pixel) of whole-image lanes against patches,
    # per workload and model; beside it the oracle's FP64 figures for the
    # same layouts if tests/golden/patch_cost.json holds them
    patch_cost = {}
    models_pc = {"B": m}
    tpath = os.path.join(ROOT, "tests", "golden", "model_b_trained.nlxw")
    if os.path.exists(tpath):
        with open(tpath, "rb") as f:
            models_pc["B_trained"] = nx.Model(f.read())
    layouts = {"whole": None, f"{ph}x{pw}": patch, "86x64": (86, 64), "64x64": (64, 64), "32x32": (32, 32)}
    wl = {"large6": ts, "uneven64": [torch.from_numpy(i).to(dev) for i in synth.workload_images("uneven64")]}
    for mname, mm in models_pc.items():
        for wname, wts in wl.items():
            wpx = sum(int(t.shape[0]) * int(t.shape[1]) for t in wts)
            rec = {}
            for lname, lp in layouts.items():
                _, ideal_img = mm.debug_symbols(wts, patch=lp)
                rec[lname] = {"qbits_per_dim": float(ideal_img.sum()) / (3 * wpx)}
            for lname in rec:
                rec[lname]["cost_vs_whole"] = rec[lname]["qbits_per_dim"] / rec["whole"]["qbits_per_dim"] - 1.0
            patch_cost.setdefault(mname, {})[wname] = rec
            log(f"[bench] patch cost, model {mname}, {wname}: " + ", ".join(
                f"{k} {v['qbits_per_dim']:.4f} ({100 * v['cost_vs_whole']:+.2f}%)" for k, v in rec.items()))
    del wl
    opath = os.path.join(ROOT, "tests", "golden", "patch_cost.json")
    if os.path.exists(opath):
        with open(opath) as f:
            patch_cost["oracle"] = json.load(f)["results"]

    for rec in whole_rec.values():
        rec["speedup_vs_raster_1024"] = raster_full_s / (rec["one_1024_ms"] / 1e3)
    out = {
        "metric": "decoded pixels/sec on 1 GPU, wavefront+patch vs raster; bits/dim gap vs FP64 oracle",
        "value": value,
        "unit": "decoded px/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "4x1024x1024 + 2x2048x1536 RGB uint8 (smooth field sigma 4, 20 edges, +-3 noise); "
                        "h=3 local model, 64 channels, 2 residual blocks, 10-logistic mixture; "
                        f"wavefront order, {pname} patches (rows x cols), one rANS lane each "
                        f"with {args.interleave} interleaved stream(s); {args.layout} decoder layout",
            "pixels": npx,
            "patch": [ph, pw],
            "interleave": args.interleave,
            "layout": args.layout,
        },
        "raster_px_per_s": raster_pxs,
        "raster_1024_s_extrapolated": raster_full_s,
        "raster_sample": f"{rows}x1024 strip, raster order, one lane, scaled by 1024/{rows}",
        "one_1024_wavefront_patch_s": one_s,
        "whole_image_row_streams": whole_rec,
        "speedup_vs_raster_1024": raster_full_s / one_s,
        "batch_px_per_s_vs_raster": value / raster_pxs,
        "encode_s_untimed": enc_s,
        "encode": enc_rec,
        "sampling": smp_rec,
        "variants": variants,
        "other_workloads": workloads,
        "other_layout_decode": alt_rec,
        "bits_per_dim": bpd,
        "gap_vs_oracle_ideal": gap,
        "roofline": {"bound": "mfma", "kernel": f"k_decode<{dims['h']},{dims['C']},false,{args.interleave},false,"
                                                 f"{'true' if args.layout == 'sheared' else 'false'}>",
                     "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "flop_per_px": flops_per_px,
                     "traffic": decode_traffic_bytes(args.layout, patch, args.interleave),
                     "traffic_unit": "HBM bytes per launch"},
        "cpu_baseline": cpu,
        "training": train_rec,
        "trained_model": trained_rec,
        "patch_bpd_cost": patch_cost,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
