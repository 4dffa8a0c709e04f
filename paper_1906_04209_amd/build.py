"""Build libnce.so (HIP kernels for gfx950 + host C++) in-tree.

Host-only C++ (precompute, tree build) is compiled by g++ with OpenMP; the
.hip sources by hipcc for gfx950; hipcc links the shared library.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
CSRC = PKG / "csrc"
OUT = PKG / "libnce.so"
BUILD = PKG / "_build"

HIP_SOURCES = ["kernels.hip", "gemm.hip", "api.hip", "batch.hip", "tree.hip", "mlp.hip", "coarse.hip", "deflate.hip", "field.hip", "precompute_gpu.hip", "types.hip"]
CPP_SOURCES = ["precompute.cpp", "tree_build.cpp", "features.cpp", "deflate_basis.cpp"]

HIPCC_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument"]
GXX_FLAGS = ["-O3", "-std=c++17", "-fPIC", "-fopenmp", "-march=x86-64-v3"]
# The far-field matrix-core kernels feed each MFMA result straight into VALU
# work; with the accumulators in AGPRs every tile pays 16 accvgpr moves.
SOURCE_FLAGS = {"tree.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r.stdout


RATES = PKG / "valu_rates"   # instruction issue-cost probe (built on request only, by build_rates)


def build(verbose: bool = False) -> Path:
    BUILD.mkdir(exist_ok=True)
    hipcc = _hipcc()
    inc = ["-I", str(CSRC), "-I", str(PKG.parent / "include")]
    jobs = []
    objs = []
    for src in CPP_SOURCES:
        o = BUILD / (Path(src).stem + ".o")
        jobs.append(["g++", *GXX_FLAGS, *inc, "-c", str(CSRC / src), "-o", str(o)])
        objs.append(str(o))
    for src in HIP_SOURCES:
        o = BUILD / (Path(src).stem + ".hip.o")
        jobs.append([hipcc, *HIPCC_FLAGS, *SOURCE_FLAGS.get(src, []), *inc,
                     "-c", str(CSRC / src), "-o", str(o)])
        objs.append(str(o))
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(_run, jobs))
    tmp = OUT.with_suffix(".so.tmp")
    _run([hipcc, "-shared", "--offload-arch=gfx950", "-fPIC", *objs, "-o", str(tmp), "-lgomp"])
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


RSQ_CHECK = PKG / "rsq_check"   # accuracy of the FP64 rsq estimate and its corrections (on request)


def build_rates() -> Path:
    """The instruction issue-cost microbenchmark and the rsq accuracy check
    (not part of the library): python -m paper_1906_04209_amd.build --rates"""
    _run([_hipcc(), *HIPCC_FLAGS, str(CSRC / "valu_rates.hip"), "-o", str(RATES)])
    _run([_hipcc(), *HIPCC_FLAGS, str(CSRC / "rsq_check.hip"), "-o", str(RSQ_CHECK)])
    return RATES


if __name__ == "__main__":
    if "--rates" in sys.argv:
        print("built", build_rates())
    else:
        build(verbose=True)
