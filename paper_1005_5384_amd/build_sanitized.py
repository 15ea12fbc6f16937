"""Sanitizer build of the library's host C++ for checks on the CPU.

The host sources (argument checks, the FP64 tree build, ownership and error
paths of the C ABI) are compiled with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and linked with the regular build's device objects
into ``libocgrav_asan.so``.  Only host-only handles (OCTGRAV_BUILD_HOST_ONLY)
and the argument checks that precede any HIP call are meant to run with it;
the device code is not instrumented.  Load it into a Python process with the
sanitizer runtimes preloaded (see ``sanitizer_env``) and OCTGRAV_LIB set to
its path.
"""
from __future__ import annotations

import os
import subprocess

from . import build as B

LIB = os.path.join(B.HERE, "libocgrav_asan.so")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined",
       "-fno-omit-frame-pointer"]


def build(verbose: bool = False) -> str:
    dev_objs = [os.path.join(B.BUILD, s + ".o") for s in B.HIP_SOURCES]
    if not all(os.path.exists(o) for o in dev_objs):
        B.build(verbose=verbose)
    host_objs = []
    for s in B.CPP_SOURCES:
        o = os.path.join(B.BUILD, s + ".asan.o")
        cxx = [f for f in B.CXX_FLAGS if f != "-O3"]
        B._run(["g++", *cxx, "-O1", "-g", *SAN, *B.INCLUDES, "-c", os.path.join(B.CSRC, s), "-o", o],
               verbose)
        host_objs.append(o)
    tmp = LIB + ".tmp"
    B._run(["g++", "-shared", "-fPIC", *SAN, "-o", tmp, *host_objs, *dev_objs, "-fopenmp",
            f"-L{B.ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{B.ROCM}/lib"], verbose)
    os.replace(tmp, LIB)
    return LIB


def sanitizer_env(base=None) -> dict:
    """Environment for a child Python process that loads the sanitized
    library: the sanitizer runtimes preloaded (they must come first), leak
    checking off (the interpreter itself keeps memory until exit), any
    report fatal."""
    env = dict(os.environ if base is None else base)
    rt = [subprocess.run(["g++", f"-print-file-name={n}"], capture_output=True, text=True,
                         check=True).stdout.strip() for n in ("libasan.so", "libubsan.so")]
    env["LD_PRELOAD"] = " ".join(rt)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    env["OCTGRAV_LIB"] = LIB
    return env


if __name__ == "__main__":
    print(build(verbose=True))
