"""Builds libspx.so (HIP for gfx950 + host C++) in the package directory."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libspx.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["graph.cpp", "runtime.cpp", "server.cpp", "spx_kernels.hip"]
# -packed-fp32-ops: keep the compiler from emitting packed FP32 VALU instructions.
# -amdgpu-mfma-vgpr-form: matrix-core accumulators in ordinary VGPRs.  Without it the FP64
# tile product keeps its accumulators in AGPRs inside the K loop but in VGPRs across the
# loop's back edge, copying all 128 of them twice per 32-deep chunk, and the out-of-line
# task bodies save more callee-saved registers to scratch.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-amdgpu-mfma-vgpr-form"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose=False):
    objs = []
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(PKG, "_build", src + ".o")
        cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
        if src.endswith(".hip"):
            cmd[1:1] = DEVICE_FLAGS
        else:
            cmd[1:1] = ["-D__HIP_PLATFORM_AMD__", "-pthread"]
        if verbose:
            print(" ".join(cmd))
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("compile failed: " + src)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *DEVICE_FLAGS, "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
