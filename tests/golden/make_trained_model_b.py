"""Writes model_b_trained.nlxw: model B after the training recipe, trained on
the CPU with the oracle's FP64 torch formulation of the code length.

Model B (h = 3, C = 64, two residual blocks, seed 12) is trained by Adam (lr
1e-3) for 2000 steps on the mean continuous code length (Eq. 2) of 64 random
32x32 crops per step, drawn from a pool of 512 smooth 64x64 images (seeds
5,000,000 + n, crops from PCG64(5,999,999)). The result, about 3-4 bits/dim on
the benchmark workloads, is the low-bits/dim model on which coded bits are
compared with the oracle's ideal. It is an input shared by both sides: it
comes from oracle/ only (not from the library's own training kernels), so
no oracle input depends on the GPU path.

Usage: python tests/golden/make_trained_model_b.py [steps]   (about 20 min on 8 cores)
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import torch_ref  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "model_b_trained.nlxw")


def main(steps: int = 2000) -> None:
    d = synth.MODEL_DIMS["B"]
    h, C, nb = d["h"], d["C"], d["n_blocks"]
    p = torch.nn.Parameter(torch.from_numpy(synth.init_params(h, C, nb, d["seed"]).astype(np.float64)))
    opt = torch.optim.Adam([p], lr=1e-3)
    pool = synth.training_pool(n=512)
    rng = np.random.Generator(np.random.PCG64(5_999_999))
    t0 = time.time()
    for step in range(steps):
        x = torch.from_numpy(synth.training_crops(pool, 64, 32, rng))
        opt.zero_grad(set_to_none=True)
        loss = torch_ref.nll_bits(p, h, C, nb, x).sum() / x.numel()
        loss.backward()
        opt.step()
        if step % 100 == 0 or step == steps - 1:
            print(f"step {step}: {float(loss.detach()):.4f} bits/dim ({time.time() - t0:.0f} s)", flush=True)
    held = torch.from_numpy(synth.training_pool(n=64, seed_base=5_500_000))
    with torch.no_grad():
        bpd = float(torch_ref.nll_bits(p, h, C, nb, held).sum()) / held.numel()
    print(f"held-out bits/dim {bpd:.4f}")
    with open(OUT, "wb") as f:
        f.write(synth.write_blob(h, C, nb, p.detach().numpy().astype(np.float32)))
    print(OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 2000)
