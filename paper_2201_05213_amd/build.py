"""Build libnellox.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libnellox.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("nx_kernels.hip", "nx_train.hip", "nx_capi.cpp")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # one rounding per operation, in source order: the encoder and the decoder
    # must produce bit-identical CDFs
    "-ffp-contract=off",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]

# flags of single sources: the coder's kernels are bound by SIMD issue, and
# LLVM's iterative ILP scheduler orders their instructions with more overlap
# than the default one (the arithmetic and its order are unchanged)
SOURCE_FLAGS = {"nx_kernels.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
                "nx_train.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]}


def coder_flags() -> list:
    """The compiler flags of the coder's kernels (nx_kernels.hip)."""
    return [f for f in HIPCC_FLAGS if f != "-shared"] + SOURCE_FLAGS["nx_kernels.hip"]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    noise = "packed-fp32-ops"
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc, *[f for f in HIPCC_FLAGS if f != "-shared"], *SOURCE_FLAGS.get(os.path.basename(src), []),
               "-c", "-I", os.path.join(ROOT, "include"), "-o", obj, src]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    errors = []
    for src, pr in procs:
        out, _ = pr.communicate()
        msg = "\n".join(l for l in out.splitlines() if noise not in l and l.strip())
        if pr.returncode != 0:
            errors.append(f"{os.path.basename(src)}:\n{msg}")
        elif verbose and msg:
            print(msg, file=sys.stderr)
    if errors:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
