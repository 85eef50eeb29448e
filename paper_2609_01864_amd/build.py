"""Builds libcredit.so for gfx950: every HIP translation unit under csrc/ is
compiled with hipcc in parallel, then linked into one shared library next to
this file.  Usage: ``python -m paper_2609_01864_amd.build`` (or ``build()``)."""
from __future__ import annotations

import json
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcredit.so")
RESOURCES = os.path.join(OUT_DIR, "kernel_resources.json")  # compiler's per-kernel resource usage
ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # contract a*b+c only inside one expression: a decoded value must be the
    # same rounded FP32 number in every pass that reads it
    "-ffp-contract=on",
    # packed FP32 instructions stay off (see the design notes)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]

SOURCES = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))

# Instruction scheduling of the forward row kernels, measured on MI355X (cold
# cache, median of 15).  The scheduler's ILP-maximising strategy against the
# default: LayerNorm FP32 N = 524288 823 -> 771 us, N = 131072 201 -> 194 us,
# softmax FP32 4096 x 65536 376 -> 365 us, FP8 softmax 478 -> 466 us.  Its
# iterative ILP strategy, later, against the ILP-maximising one: LayerNorm
# FP32 N = 524288 759 -> 745 us, the other LayerNorm shapes within +-1%, so
# the FP32 / BF16 LayerNorm instances take it; for the softmax it spilled
# the LDS-slice instances (up to 2.3 KiB per lane) and slowed FP8 rows by
# 3.5%, and RMSNorm gained nothing, so those keep the ILP-maximising one.
# The backward kernels and the FP8 LayerNorm / RMSNorm forward (+1% / +2.4%
# with max-ilp, and two FP8 RMSNorm slices spill) keep the default schedule.
_MAX_ILP = ["-mllvm", "-amdgpu-sched-strategy=max-ilp"]
_ITER_ILP = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"]
FILE_FLAGS = {"inst_ln_fwd.hip": _ITER_ILP, "inst_softmax_fwd.hip": _MAX_ILP, "inst_rms_fwd.hip": _MAX_ILP}


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]"
                     r"|VGPRs Spill|LDS Size \[bytes/block\]): (\S+)")
_KEYS = {"VGPRs": "vgprs", "AGPRs": "agprs", "ScratchSize [bytes/lane]": "scratch_bytes",
         "Occupancy [waves/SIMD]": "waves_per_simd", "VGPRs Spill": "vgpr_spills", "LDS Size [bytes/block]": "lds_bytes"}


def _resources(stderr: str) -> dict:
    """Per-kernel resource usage from the compiler's kernel-resource-usage
    remarks (registers, private bytes per lane, waves per SIMD, LDS)."""
    out, cur = {}, None
    for m in _REMARK.finditer(stderr):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = int(val)
    return out


def _compile(src: str):
    obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), "-Rpass-analysis=kernel-resource-usage", "-I", CSRC, "-c",
           os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-x")
        cmd.insert(2, "hip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    return obj, _resources(r.stderr)


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(jobs) as ex:
        done = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in done]
    res = {}
    for _, r in done:
        res.update(r)
    with open(RESOURCES, "w") as f:
        json.dump(res, f, indent=0, sort_keys=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(SOURCES)} sources", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
