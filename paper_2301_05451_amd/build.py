"""Build ``libtq.so`` for gfx950 with hipcc (objects compiled in parallel, then linked).

Usage: ``python -m paper_2301_05451_amd.build`` (always recompiles).

``python -m paper_2301_05451_amd.build --host-sanitize`` builds ``_build_san/libtq_san.so``
instead: host code built with AddressSanitizer and UndefinedBehaviorSanitizer (device code
is built as usual and not instrumented), for checking the host-side planners on the CPU (the
state-vector schedule builder, the tensor-network plan builder, gate lowering, Pauli
decomposition) on the CPU. Load it with ``TQ_LIBRARY`` set to its path and clang's ASan
runtime preloaded (``sanitizer_runtime()``).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtq.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["api.hip", "schedule.hip", "sv_kernels.hip", "expval.hip", "sv_adjoint.hip", "tn.hip", "mlp.hip", "batched.hip", "observables.hip", "optim.hip", "peaks.hip"]

# Packed FP32 instructions are disabled for device code (the host pass warns that it does
# not know the feature; that is harmless). Matrix-core instructions take their accumulators
# in ordinary vector registers: with the default accumulation-register form the compiler
# copied every accumulator into and out of those registers around each k-step of the
# complex GEMMs (64 copies per 16 FP64 MFMAs), and a bare MFMA loop reached 63 % of the FP64
# rate instead of 99 %. Kernels without matrix-core instructions compile to the same code.
MFMA_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *MFMA_FLAGS,
    "-I", os.path.join(ROOT, "include"),
]


SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_OBJ, "libtq_san.so")
# every -fsanitize= goes to the host pass only
SAN_FLAGS = [
    "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *MFMA_FLAGS, "-O1", "-g",
    "-fno-omit-frame-pointer", "-std=c++17",
    "-fPIC", "-Wno-unused-function", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
]


def sanitizer_runtime():
    """Path of clang's shared AddressSanitizer runtime that the sanitized library needs."""
    base = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "llvm", "lib", "clang")
    for ver in sorted(os.listdir(base), reverse=True) if os.path.isdir(base) else []:
        p = os.path.join(base, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise RuntimeError("clang's ASan runtime (libclang_rt.asan-x86_64.so) not found")


def build_sanitized():
    os.makedirs(SAN_OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def one(src):
        obj = os.path.join(SAN_OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc(), *SAN_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(one, srcs))
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-shared-libsan", "-o", SAN_LIB, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return SAN_LIB


def hipcc():
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def _compile(src):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    if "--host-sanitize" in sys.argv:
        print(build_sanitized())
    else:
        print(build(verbose="-v" in sys.argv))
