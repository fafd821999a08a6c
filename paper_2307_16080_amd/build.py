"""Build the HIP library ``libmlk.so`` for gfx950 in-tree, and the OpenMP
host-kernel library ``libmlkhost.so``.

Every source under ``csrc/`` is compiled by hipcc to an object file in
``_build/`` (in parallel), then linked into ``libmlk.so`` next to this file.
The C ABI is declared in ``include/mlk.h`` at the repository root; the host
kernels' in ``include/mlk_host.h``.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmlk.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -packed-fp32-ops: no packed fp32 VALU instructions in any kernel.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]

SOURCES = ["k_f32.hip", "k_bf16.hip", "k_fast.hip", "k_i8.hip", "k_f8.hip", "k_conv.hip", "k_conv_f32.hip", "k_direct.hip", "elementwise.hip", "probe.hip",
           "mlp.hip", "api.cpp", "batched.cpp", "conv_batch.cpp", "tune.cpp", "model.cpp", "scratch.cpp"]


def _compile(src: str, verbose: bool) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC] + FLAGS + lang + ["-c", path, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    if err.strip() and verbose:
        print(err, file=sys.stderr)
    return obj


HOST_SRC = os.path.join(HERE, "host", "mlk_host.cpp")
HOST_LIB = os.path.join(HERE, "libmlkhost.so")


def build_host(verbose: bool = False) -> str:
    """The OpenMP host kernels (include/mlk_host.h) as their own library,
    libmlkhost.so: g++, no HIP, nothing shared with libmlk.so."""
    cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-mavx2", "-mfma", "-fPIC", "-shared", "-Wall",
           HOST_SRC, "-o", HOST_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(HOST_LIB + ".tmp", HOST_LIB)
    return HOST_LIB


def build(verbose: bool = False, jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, len(os.sched_getaffinity(0))))
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    build_host(verbose)
    return LIB


if __name__ == "__main__":
    t = build(verbose="-v" in sys.argv)
    print(t)
