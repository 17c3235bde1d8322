"""Build the HIP library libapic.so in-tree for gfx950.

    python -m paper_2407_20469_amd.build          # or build() from Python

hipcc compiles the kernels and the C ABI (csrc/api.hip) and the host plan
builder (csrc/plan.cpp) into one shared library next to this file.  Packed
FP32 instructions are disabled for all device code.
"""

import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libapic.so")
ARCH = os.environ.get("APIC_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.hip", "plan.cpp"]
HEADERS = ["common.hpp", "fft.hpp", "zern.hpp", "kernels_bf.hpp", "kernels_df.hpp", "chol.hpp",
           "calib.hpp", "plan.hpp"]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the APIC library needs ROCm's hipcc to build")


def command(out=LIB):
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument", "-I", INCLUDE,
            *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(verbose=True):
    """Compile libapic.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    t0 = time.time()
    if verbose:
        print("[apic build]", " ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[apic build] {LIB} ({time.time() - t0:.1f} s)", flush=True)
    return LIB


if __name__ == "__main__":
    build()
