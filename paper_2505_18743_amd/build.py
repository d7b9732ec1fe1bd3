"""Build the gfx950 shared library libswdg.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libswdg.so")

SOURCES = ["sw_api.hip", "sw_ens.hip", "sw_setup.hip", "sw_face.hip", "sw_stage_r1.hip", "sw_stage_r2.hip",
           "sw_stage_r3.hip", "sw_tracer_r1.hip", "sw_tracer_r2.hip", "sw_tracer_r3.hip", "sw_vjp_r1.hip", "sw_vjp_r2.hip", "sw_vjp_r3.hip", "sw_vjp_face.hip", "sw_amr.hip", "sw_react.hip"]
ARCH = "gfx950"
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         # multiply-adds fuse where the source writes them as one expression,
         # the same in every kernel that inlines a shared helper
         "-ffp-contract=on",
         # packed FP32 instructions stay off (FP64 library; hipcc's host pass warns, harmless)
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", INCLUDE, "-I", CSRC, "-Wno-unused-command-line-argument"]


def _hipcc():
    for cand in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(cand) or cand == "hipcc":
            return cand
    return "hipcc"


def _compile(src, jobs_env):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc()] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True, env=jobs_env)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
    return obj


def build_library(jobs: int | None = None) -> str:
    """Compile every HIP source for gfx950 and link libswdg.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    env = dict(os.environ)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 2) - 1), 6)
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, env), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library())
