"""Build libqaoa.so (HIP kernels + host runtime behind include/qaoa.h) for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqaoa.so")
SOURCES = ["qaoa_kernels.hip", "qaoa_xpass.hip", "qaoa_swz_f32.hip", "qaoa_swz_f64.hip", "qaoa_clique.hip",
           "qaoa_grover.hip", "qaoa_xmix.hip",
           "qaoa_gemm.hip", "qaoa_api.cpp", "qaoa_angles.cpp"]
HOST_ONLY = {"qaoa_angles.cpp"}  # plain C++ above the C ABI: no device code
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are disabled for every HIP source of this library.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument"]


def _stale(obj: str, src: str) -> bool:
    """True when the object is missing or older than its source or any header it may include."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(ROOT, "include", "qaoa.h"))
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, jobs: int = 4, force: bool = True) -> str:
    """Compile every source to an object (in parallel; with force=False only the objects older
    than their sources or headers), then link the shared library."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        objs.append(obj)
        if not force and not _stale(obj, src):
            continue
        lang = ["-x", "hip"] if src.endswith(".cpp") and src not in HOST_ONLY else []
        omp = ["-fopenmp"] if src in HOST_ONLY else []  # the optimiser's per-run updates
        cmd = [HIPCC] + FLAGS + lang + omp + ["-I", os.path.join(ROOT, "include"), "-c",
                                              os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        while len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out = p.communicate()[0].decode(errors="replace")
        lines = [l for l in out.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-fopenmp", "-o", tmp] + objs + \
          ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/llvm/lib"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="--changed" not in sys.argv))
