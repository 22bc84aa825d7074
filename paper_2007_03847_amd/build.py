"""Build libfmc.so (all HIP sources, gfx950) in the package directory.

Every source is compiled by hipcc for gfx950 in parallel and linked into one
shared library exporting the C ABI of include/fmc.h.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfmc.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
SOURCES = ["fmc_runtime.hip", "fmc_run.hip", "fmc_fd.hip", "fmc_batch.hip", "fmc_serve.hip", "k_decor.hip", "k_rrf.hip",
           "k_sample.hip", "k_setup.hip", "k_fluxdecay.hip", "k_batch.hip", "k_mfma_classical.hip",
           "k_integrate_f64.hip", "k_integrate_f32.hip", "k_integrate_gen_f64.hip",
           "k_integrate_gen_f32.hip", "k_trap.hip"]
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# Per-source flags.  The KLE contractions keep their accumulators in the
# matrix-operation form that reads and writes ordinary vector registers, so
# the loop carries no copies between them and the accumulation registers.
SOURCE_FLAGS = {"k_sample.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=1"]}


def _newest_header() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))]
    hs.append(os.path.join(HERE, "..", "include", "fmc.h"))
    return max(os.path.getmtime(h) for h in hs if os.path.exists(h))


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    if incremental and os.path.exists(obj):
        t = os.path.getmtime(obj)
        if t > os.path.getmtime(os.path.join(CSRC, src)) and t > _newest_header():
            return obj
    cmd = [HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, incremental: bool = False) -> str:
    """Compile every source (incremental: only those older than their
    source or any header) and link the library."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda f: _compile(f, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--incremental"]
    print(build(int(args[0]) if args else None, incremental="--incremental" in sys.argv))
