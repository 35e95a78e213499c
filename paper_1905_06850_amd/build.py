"""Build libplcg.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libplcg.so")
SOURCES = [os.path.join(HERE, "csrc", "plcg_kernels.hip"),
           os.path.join(HERE, "csrc", "plcg_var_kernels.hip"),
           os.path.join(HERE, "csrc", "plcg_resident.hip"),
           os.path.join(HERE, "csrc", "plcg_batch_kernels.hip"),
           os.path.join(HERE, "csrc", "plcg_noalloc.hip"),
           os.path.join(HERE, "csrc", "plcg_engine.cpp"),
           os.path.join(HERE, "csrc", "plcg_batch.cpp"),
           os.path.join(HERE, "csrc", "plcg_serve.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for every HIP translation unit.  No
# floating-point contraction: every fused multiply-add is an fma() in the source,
# so a value's roundings follow from the source alone, whatever the compiler
# schedules (the same in every kernel and code path that computes it).
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
         "-Wall", "-Wno-unused-command-line-argument",
         "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose, what):
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError(f"hipcc failed {what}")
    if verbose and proc.stderr.strip():
        sys.stderr.write(proc.stderr)


def build(verbose: bool = False) -> str:
    """Compile the translation units in parallel (each holds its own device
    code; no relocatable device code), then link them into libplcg.so."""
    tmp = LIB + ".tmp"
    compile_flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="plcg_build_") as d:
        objs = [os.path.join(d, os.path.basename(src) + ".o") for src in SOURCES]
        jobs = [([HIPCC, *compile_flags, "-c", src, "-o", obj], f"compiling {src}")
                for src, obj in zip(SOURCES, objs)]
        workers = max(1, min(len(jobs), os.cpu_count() or 1))
        with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
            for f in [ex.submit(_run, cmd, verbose, what) for cmd, what in jobs]:
                f.result()
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose,
             "linking libplcg.so")
    os.replace(tmp, LIB)
    return LIB


C_EXAMPLE = os.path.join(ROOT, "tests", "c", "solve_file.c")
C_EXAMPLE_BIN = os.path.join(ROOT, "tests", "c", "solve_file")


def build_c_caller(verbose: bool = False) -> str:
    """The plain C caller used by the tests (host code only, linked to libplcg.so)."""
    cmd = [HIPCC, "-x", "hip", *[f for f in FLAGS if f not in ("-fPIC", "-shared")], C_EXAMPLE,
           "-o", C_EXAMPLE_BIN + ".tmp", "-L", HERE, "-lplcg",
           "-Wl,-rpath,$ORIGIN/../../" + os.path.basename(HERE)]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        sys.stderr.write(proc.stdout + proc.stderr)
        raise RuntimeError("hipcc failed building the C caller")
    os.replace(C_EXAMPLE_BIN + ".tmp", C_EXAMPLE_BIN)
    return C_EXAMPLE_BIN


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_c_caller(verbose=True))
