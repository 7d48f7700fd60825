"""Build libmd.so (HIP for gfx950) in-tree with hipcc.

``python -m paper_2606_08039_amd.build`` or ``build.build()``.  Every call
compiles; nothing is cached.  All device code is compiled with packed FP32
instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmd.so")

HIP_SOURCES = ["md_step.hip", "md_step_dr.hip", "md_step_wind.hip", "md_rk4.hip", "md_mlp.hip", "md_surrogate.hip"]
CPP_SOURCES = ["md_api.cpp", "md_tune.cpp"]

ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
# per-source options: the surrogate step keeps its MFMA accumulators in
# ordinary VGPRs, so that the SiLU epilogue reads them without a copy out of
# the accumulation registers
EXTRA = {"md_surrogate.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False, jobs=8):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs, procs = [], []
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc, "-x", "hip", "-c"] + COMMON + DEVICE + EXTRA.get(src, []) + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    for src in CPP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [hipcc, "-c"] + COMMON + DEVICE + [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    bad = [src for p, src in procs if p.wait() != 0]
    if bad:
        raise RuntimeError("hipcc failed for: " + ", ".join(bad))
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
