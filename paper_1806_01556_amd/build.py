"""Build libfdas.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1806_01556_amd.build   (or call build()).
Every HIP and C++ source under csrc/ is compiled into one shared library next
to this file.  Packed-FP32 instructions are disabled for all device code.
"""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfdas.so")
ARCH = os.environ.get("FDAS_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp"))
    )


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    out_tmp = LIB + ".tmp"
    cmd = [
        hipcc(),
        "-std=c++17",
        "-O3",
        "-fPIC",
        "-shared",
        f"--offload-arch={ARCH}",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-fno-slp-vectorize",
        "-Wno-unused-command-line-argument",
        "-I", os.path.join(os.path.dirname(HERE), "include"),
        "-pthread",
        "-o", out_tmp,
    ] + sources()
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}")
    warn = "\n".join(
        l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip()
    )
    if verbose and warn:
        print(warn)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
