"""Build libgm.so (the HIP kernels and the C ABI of include/gm.h) for gfx950, in-tree.

Every source is compiled with hipcc for gfx950 only.  Packed FP32 instruction selection is
disabled on every device pass.  The box/record kernel is compiled without floating-point
contraction (its integer boxes follow one exact IEEE binary64 recipe).

The build also records, in kernel_digests.json beside the library, the SHA-256 of the gfx950
assembly of the kernels whose hardware counters are kept as summaries: a summary applies to a
build exactly when the digest it was taken with is still the one recorded here.
"""
from __future__ import annotations

import concurrent.futures as cf
import hashlib
import json
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgm.so")

SOURCES = ["gm_api.hip", "preprocess.hip", "binning.hip", "render.hip", "backward.hip",
           "optim.hip", "init.hip", "nrf.hip", "nrf_fwd.hip", "warm.hip", "ssim.hip"]
NO_CONTRACT = {"preprocess.hip"}
# MFMA results in ordinary VGPRs rather than AGPRs: the field's forward reads every accumulator
# back for the activation, which AGPRs would cost one v_accvgpr_read each (the field's chain
# kernel, in nrf.hip, holds more live registers and runs 3% slower so built)
MFMA_VGPR = {"nrf_fwd.hip"}

COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
          "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I" + os.path.join(ROOT, "include")]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _flags(src: str) -> list:
    flags = list(COMMON)
    if src in NO_CONTRACT:
        flags.append("-ffp-contract=off")
    if src in MFMA_VGPR:
        flags += ["-mllvm", "-amdgpu-mfma-vgpr-form"]
    return flags


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    flags = _flags(src)
    cmd = [hipcc()] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


# kernels with counter summaries (profiles/<kernel>_traffic_*.md): source file and the
# kernel's symbol as it appears mangled (the instantiation the benchmark runs)
DIGESTED = {"k_partials": ("backward.hip", "10k_partialsILb0E"),
            "k_render": ("render.hip", "8k_renderE")}
DIGESTS = os.path.join(HERE, "kernel_digests.json")


def _kernel_asm_digest(src: str, kernels) -> dict:
    """SHA-256 of each kernel's gfx950 assembly (its function body, labels included);
    kernels maps a name to its mangled symbol fragment."""
    flags = _flags(src)
    out = os.path.join(BUILD, os.path.splitext(src)[0] + ".s")
    cmd = [hipcc()] + flags + ["--cuda-device-only", "-S", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"assembly of {src} failed:\n{r.stderr}")
    with open(out) as f:
        lines = f.read().splitlines()
    res = {}
    for k, tag in kernels.items():
        body, inside = [], False
        for ln in lines:
            head = ln.split(";")[0].strip()
            if not inside and head.endswith(":") and tag in head and not head.startswith("."):
                inside = True
            if inside:
                body.append(ln)
                if ln.startswith(".Lfunc_end"):
                    break
        if body:
            res[k] = hashlib.sha256("\n".join(body).encode()).hexdigest()
    return res


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    by_src = {}
    for k, (src, tag) in DIGESTED.items():
        by_src.setdefault(src, {})[k] = tag
    with cf.ThreadPoolExecutor(max_workers=len(by_src)) as ex:
        parts = list(ex.map(lambda kv: _kernel_asm_digest(*kv), by_src.items()))
    digests = {k: v for d in parts for k, v in d.items()}
    with open(DIGESTS, "w") as f:
        json.dump(digests, f, indent=1, sort_keys=True)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
