"""Build libsyk.so in-tree: host C++ with g++, HIP kernels with hipcc for gfx950.

Usage: python paper_2311_00639_amd/build.py [-v]  (or __graft_entry__.build())."""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsyk.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["terms.cpp", "runtime.cpp", "apply_plan.cpp", "krylov.cpp", "otoc.cpp", "engine.cpp", "batch.cpp", "op.cpp", "analysis.cpp", "otoc_ensemble.cpp", "api.cpp"]
HIP_SOURCES = ["kernels.hip", "apply_tiled.hip", "batch.hip"]

HOST_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall", "-Wextra", "-Wno-unused-parameter",
              "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-I" + CSRC,
              # one IEEE operation at a time: the coupling draws must round as written
              "-ffp-contract=off"]
HIP_FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-I" + CSRC,
             # packed FP32 instructions are disabled on this target
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-munsafe-fp-atomics"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if p.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + p.stdout)
        raise RuntimeError("build step failed: " + cmd[-1])
    return p.stdout


def build(verbose: bool = False) -> str:
    """Compile every source and link libsyk.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        jobs.append([hipcc] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj])
    procs = [(j, subprocess.Popen(j, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)) for j in jobs]
    failed = []
    for cmd, p in procs:
        out, _ = p.communicate()
        if verbose or p.returncode != 0:
            sys.stderr.write(" ".join(cmd) + "\n" + (out or ""))
        if p.returncode != 0:
            failed.append(cmd[-3])
    if failed:
        raise RuntimeError("compilation failed: " + ", ".join(failed))
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs +
         ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
