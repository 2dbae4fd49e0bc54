"""Build libabp.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB_PATH = os.path.join(PKG, "libabp.so")

# Packed FP32 (v_pk_*_f32) is switched off for all device code: only plain VALU FP32 is emitted.
HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function"]

# Per-file additions. The stochastic Heun integrator, the adjoint's in-place forward phase and its
# Heun backward are scheduled with LLVM's AMDGPU "max-ilp" strategy (instruction-level parallelism
# first): their loops carry long dependency chains per wavefront, and it measured 1.5-2% faster
# there. The persistent batched kernel and the 16-step Euler-Maruyama backward of the exact
# gradient use "iterative-minreg": the 4096-set sweep 7% faster with the same instructions, the
# backward 4% faster at two wavefronts per SIMD (fewer spills) and 1.3% at one; the 8-step and
# the decayed estimator's backward variants measured slower under it and stay with max-ilp. The
# adjoint's forward phase with the noise look-ahead loop (the 65536-particle form) uses
# "iterative-ilp": 3.5% (Euler-Maruyama) and 2.4% (Heun) faster than under max-ilp. The
# Euler-Maruyama integrator keeps the default schedule (max-ilp and the iterative strategies
# measured 0.2-1.6% slower). The instructions are the same, only their order and register
# assignment differ.
FILE_FLAGS = {
    "integrate_heun.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "adjoint.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
    "adjoint_em.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-minreg"],
    "batched.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-minreg"],
    "adjoint_fwd.hip": ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"],
}


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the HIP library cannot be built")
    return exe


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def flags_for(src: str) -> list[str]:
    """The device-code flags one source file is compiled with (no -shared)."""
    base = [f for f in HIPCC_FLAGS if f != "-shared"]
    return base + FILE_FLAGS.get(os.path.basename(src), [])


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB_PATH) -> str:
    """Compile every source with its flags (in parallel), then link libabp.so."""
    srcs = sources()
    objdir = tempfile.mkdtemp(prefix="abp_build_")
    try:
        def compile_one(src: str) -> str:
            obj = os.path.join(objdir, os.path.basename(src) + ".o")
            cmd = [hipcc(), *flags_for(src), *(extra or []), "-c", src, "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            res = subprocess.run(cmd, capture_output=True, text=True)
            if res.returncode != 0:
                raise RuntimeError("hipcc failed on " + src + ":\n" + res.stdout + res.stderr)
            return obj

        with ThreadPoolExecutor(min(len(srcs), 8)) as pool:
            objs = list(pool.map(compile_one, srcs))
        tmp = out + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, out)
    finally:
        shutil.rmtree(objdir, ignore_errors=True)
    return out


UBENCH_SRC = os.path.join(PKG, "ubench", "valu_rates.hip")
UBENCH_BIN = os.path.join(PKG, "ubench", "valu_rates")


def build_ubench(verbose: bool = False) -> str:
    """The VALU issue-rate microbenchmark behind the roofline denominators (a standalone binary)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    cmd = [hipcc(), *flags, UBENCH_SRC, "-o", UBENCH_BIN]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    return UBENCH_BIN


ROOT = os.path.dirname(PKG)
CLIENT_SRC = os.path.join(ROOT, "tests", "c_client", "abi_client.cpp")
CLIENT_BIN = os.path.join(ROOT, "tests", "c_client", "abi_client")


def build_client(verbose: bool = False) -> str:
    """A host program that uses libabp through include/abp.h alone (the C ABI test client); it
    finds libabp.so through an rpath relative to itself."""
    cmd = [hipcc(), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), CLIENT_SRC,
           "-L", PKG, "-labp", "-Wl,-rpath,$ORIGIN/../../paper_1104_2499_amd", "-o", CLIENT_BIN]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    return CLIENT_BIN


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_ubench(verbose=True))
    print(build_client(verbose=True))
