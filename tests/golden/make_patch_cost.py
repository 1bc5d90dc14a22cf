"""Writes patch_cost.json: the oracle's quantised-ideal code length of the
benchmark workloads with whole-image lanes and with patches, per model.

The patch scheme codes every patch as an independent image: context across
patch borders is zero, so patches cost bits against whole-image coding, the
paper's exact method (Sec. 4 and Table 2 report the same bits/dim for every
decoder of one image). For large6 (4 x 1024^2 + 2 x 2048x1536) and uneven64
(64 images of uneven sizes) this computes, with the FP64 oracle over every
pixel, the quantised ideal -sum log2(f / 2^16) for whole-image lanes and for
86x64 (the benchmark's patches on 256 CUs), 64x64 and 32x32 patches, for the
random-init model B and for the trained model B (model_b_trained.nlxw).

Usage: python tests/golden/make_patch_cost.py [processes]   (about 15 min on 8 cores)
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

LAYOUTS = {"whole": (0, 0), "86x64": (86, 64), "64x64": (64, 64), "32x32": (32, 32)}
WORKLOADS = ("large6", "uneven64")


def model_blobs():
    import synth

    with open(os.path.join(HERE, "model_b_trained.nlxw"), "rb") as f:
        trained = f.read()
    return {"B": synth.model_blob("B")[0], "B_trained": trained}


def job(args):
    mname, wname, k, layout = args
    import oracle
    import synth

    img = synth.workload_images(wname, count=1, start=k)[0]
    om = oracle.Model.from_blob(model_blobs()[mname])
    ph, pw = LAYOUTS[layout]
    t = time.time()
    s = om.stats(img, ph, pw)
    return mname, wname, k, layout, s["qbits"], s["cbits"], img.shape[0] * img.shape[1], time.time() - t


def main(procs: int) -> None:
    import synth

    jobs = []
    for mname in ("B", "B_trained"):
        for wname in WORKLOADS:
            for k in range(len(synth.workload_shapes(wname))):
                for layout in LAYOUTS:
                    jobs.append((mname, wname, k, layout))
    # largest images first, so the pool ends together
    jobs.sort(key=lambda j: -synth.workload_shapes(j[1])[j[2]][0] * synth.workload_shapes(j[1])[j[2]][1])
    out = {}
    t0 = time.time()
    with mp.get_context("spawn").Pool(procs) as pool:
        for n, (mname, wname, k, layout, q, c, npx, dt) in enumerate(pool.imap_unordered(job, jobs)):
            r = out.setdefault(mname, {}).setdefault(wname, {}).setdefault(layout, {"qbits": 0.0, "cbits": 0.0,
                                                                                   "pixels": 0})
            r["qbits"] += q
            r["cbits"] += c
            r["pixels"] += npx
            if n % 20 == 0:
                print(f"{n + 1}/{len(jobs)} jobs ({time.time() - t0:.0f} s)", flush=True)
    for mname, ws in out.items():
        for wname, ls in ws.items():
            whole = ls["whole"]["qbits"]
            for layout, r in ls.items():
                r["qbits_per_dim"] = r["qbits"] / (3 * r["pixels"])
                r["cost_vs_whole"] = r["qbits"] / whole - 1.0
    doc = {"what": "oracle (FP64) quantised-ideal bits -sum log2(f/2^16) and continuous bits, every pixel; "
                   "patches coded as independent images (zero context across borders)",
           "layouts": {k: list(v) for k, v in LAYOUTS.items()}, "results": out}
    with open(os.path.join(HERE, "patch_cost.json"), "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)
    for mname, ws in out.items():
        for wname, ls in ws.items():
            print(mname, wname, {l: f"{r['qbits_per_dim']:.4f} ({100 * r['cost_vs_whole']:+.3f}%)" for l, r in ls.items()})


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count() or 4)
