"""Builds libocgrav.so in-tree: HIP kernels with hipcc for gfx950, host C++
with g++ (OpenMP), linked by hipcc into one shared library."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libocgrav.so")
# measurement program: issue rate of non-packed FP32 / INT32 VALU instructions
VALU_RATE = os.path.join(HERE, "valu_rate")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_SOURCES = ["walk.hip", "eval.hip", "walk_eval.hip", "walk_eval_block.hip", "mac.hip", "mlp.hip",
               "tree_gpu.hip", "integrate.hip", "noalloc.hip"]
CPP_SOURCES = ["tree_build.cpp", "capi.cpp"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # keep IEEE FP32 denormals (the opening test is bit-exact against the host)
    "-fno-gpu-flush-denormals-to-zero",
    # matrix-core results straight in VGPRs (no accumulation-register copies)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
    "-Wall", "-Wno-unused-function",
]
CXX_FLAGS = ["-std=c++17", "-O3", "-fopenmp", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
             f"-I{ROCM}/include"]
INCLUDES = [f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build step failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r


def build(verbose: bool = False, extra_hip_flags=()) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HIP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs.append(([f"{ROCM}/bin/hipcc", *HIPCC_FLAGS, *extra_hip_flags, *INCLUDES, "-c",
                      os.path.join(CSRC, s), "-o", o], o))
    for s in CPP_SOURCES:
        o = os.path.join(BUILD, s + ".o")
        jobs.append((["g++", *CXX_FLAGS, *INCLUDES, "-c", os.path.join(CSRC, s), "-o", o], o))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    tmp = LIB + ".tmp"
    _run([f"{ROCM}/bin/hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
          *[o for _, o in jobs], "-lgomp", "-Wl,--no-undefined", f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, LIB)
    _run([f"{ROCM}/bin/hipcc", *HIPCC_FLAGS, "-o", VALU_RATE + ".tmp",
          os.path.join(CSRC, "valu_rate.hip")], verbose)
    os.replace(VALU_RATE + ".tmp", VALU_RATE)
    return LIB


def disassemble(source: str, out: str) -> None:
    """Writes the gfx950 assembly of one HIP source (for inspection)."""
    _run([f"{ROCM}/bin/hipcc", *HIPCC_FLAGS, *INCLUDES, "--cuda-device-only", "-S",
          os.path.join(CSRC, source), "-o", out], False)


if __name__ == "__main__":
    print(build(verbose=True))
