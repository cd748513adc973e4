"""Build libtpcca.so for gfx950 with hipcc (run on any machine with ROCm; no GPU
needed).  The kernel source is compiled twice: the deterministic object
(no FP contraction, correctly rounded division and square root) and the
production object (contraction, fast reciprocal)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtpcca.so")
ARCH = os.environ.get("TPC_OFFLOAD_ARCH", "gfx950")

COMMON = ["--offload-arch=" + ARCH, "-O3", "-fPIC", "-std=c++17",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC,
          # no packed FP32 instructions (v_pk_*_f32) anywhere
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]
DET = ["-DTPC_NS=det", "-DTPC_DET=1", "-ffp-contract=off",
       "-fhip-fp32-correctly-rounded-divide-sqrt"]
PROD = ["-DTPC_NS=prod", "-DTPC_DET=0", "-ffp-contract=fast",
        "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-freciprocal-math", "-fno-signed-zeros",
        "-fgpu-flush-denormals-to-zero"]
# the refit's reverse pass is held to a tolerance, not to bits
BWD = ["-ffast-math", "-fno-finite-math-only"]


def _hipcc():
    return os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = [
        ([_hipcc(), *COMMON, "-c", os.path.join(CSRC, "tpc_api.cpp"),
          "-o", os.path.join(BUILD, "tpc_api.o")], "tpc_api.o"),
        ([_hipcc(), *COMMON, "-c", os.path.join(CSRC, "tpc_prof.cpp"),
          "-o", os.path.join(BUILD, "tpc_prof.o")], "tpc_prof.o"),
        ([_hipcc(), *COMMON, *DET, "-c", os.path.join(CSRC, "tpc_kernels.hip"),
          "-o", os.path.join(BUILD, "tpc_kernels_det.o")], "tpc_kernels_det.o"),
        ([_hipcc(), *COMMON, *PROD, "-c", os.path.join(CSRC, "tpc_kernels.hip"),
          "-o", os.path.join(BUILD, "tpc_kernels_prod.o")], "tpc_kernels_prod.o"),
        ([_hipcc(), *COMMON, *DET, "-c", os.path.join(CSRC, "tpc_refit.hip"),
          "-o", os.path.join(BUILD, "tpc_refit_det.o")], "tpc_refit_det.o"),
        ([_hipcc(), *COMMON, *PROD, "-c", os.path.join(CSRC, "tpc_refit.hip"),
          "-o", os.path.join(BUILD, "tpc_refit_prod.o")], "tpc_refit_prod.o"),
        ([_hipcc(), *COMMON, *DET, "-c", os.path.join(CSRC, "tpc_transform.hip"),
          "-o", os.path.join(BUILD, "tpc_transform_det.o")], "tpc_transform_det.o"),
        ([_hipcc(), *COMMON, *PROD, "-c", os.path.join(CSRC, "tpc_transform.hip"),
          "-o", os.path.join(BUILD, "tpc_transform_prod.o")], "tpc_transform_prod.o"),
        ([_hipcc(), *COMMON, *DET, "-c", os.path.join(CSRC, "tpc_merge.hip"),
          "-o", os.path.join(BUILD, "tpc_merge_det.o")], "tpc_merge_det.o"),
        ([_hipcc(), *COMMON, *PROD, "-c", os.path.join(CSRC, "tpc_merge.hip"),
          "-o", os.path.join(BUILD, "tpc_merge_prod.o")], "tpc_merge_prod.o"),
        ([_hipcc(), *COMMON, *BWD, "-c", os.path.join(CSRC, "tpc_refit_bwd.hip"),
          "-o", os.path.join(BUILD, "tpc_refit_bwd.o")], "tpc_refit_bwd.o"),
    ]
    procs = []
    for cmd, _ in jobs:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                      text=True))
    failed = []
    for p, (cmd, name) in zip(procs, jobs):
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((name, out))
        elif verbose and out.strip():
            print(out)
    if failed:
        msg = "\n".join(f"--- {n}\n{o}" for n, o in failed)
        raise RuntimeError("hipcc failed:\n" + msg)
    tmp = LIB + ".tmp"
    subprocess.run([_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp,
                    *[os.path.join(BUILD, j[1]) for j in jobs]], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
