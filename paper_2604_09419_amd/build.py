"""Build liblinehip.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2604_09419_amd.build [--incremental]

Every translation unit under csrc/ is compiled to an object in parallel and the
objects are linked into paper_2604_09419_amd/liblinehip.so.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
SO = os.path.join(HERE, "liblinehip.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-fvisibility=hidden",
    # packed binary32 VALU ops are disabled for every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
# The alias construction must round every binary64 operation on its own.
PER_FILE = {"alias.hip": ["-ffp-contract=off"], "walk.hip": ["-ffp-contract=off"]}
# Training units: a branch on a wave-uniform condition (a row's store or atomic) stays one
# if/else instead of two guarded blocks, so the compiler knows that exactly one write
# follows each row and its waits on vmcnt cover only the loads they need.
UNIFORM_BRANCHES = ["-mllvm", "-structurizecfg-skip-uniform-regions=true"]
for _name in ("sgd_f32_o1.hip", "sgd_f32_o2.hip", "sgd_f32_o3.hip", "sgd_bf16_o1.hip", "sgd_bf16_o2.hip",
              "sgd_bf16_o3.hip", "batch.hip"):
    PER_FILE[_name] = UNIFORM_BRANCHES


def _headers_mtime() -> float:
    hs = glob.glob(os.path.join(CSRC, "*.hpp")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, incremental: bool, hdr_mtime: float) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t >= os.path.getmtime(src) and t >= hdr_mtime:
            return obj
    cmd = [HIPCC, *COMMON, *PER_FILE.get(os.path.basename(src), []), "-c", src, "-o", obj + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    os.replace(obj + ".tmp", obj)
    return obj


def build(incremental: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hdr = _headers_mtime()
    jobs = jobs or max(1, min(len(srcs), os.cpu_count() or 1, 16))
    # largest units first
    srcs.sort(key=lambda s: 0 if os.path.basename(s).startswith("sgd_") else 1)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental, hdr), srcs))
    tmp = SO + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(incremental="--incremental" in sys.argv))
