"""Build libfdas.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1806_01556_amd.build   (or call build()).
Every HIP and C++ source under csrc/ is compiled (in parallel, one object per
source under _build/) and linked into one shared library next to this file.
Packed-FP32 instructions are disabled for all device code.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

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


COMMON = [
    "-std=c++17",
    "-O3",
    "-fPIC",
    f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-slp-vectorize",
    "-Wno-unused-command-line-argument",
    "-pthread",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with exit code {res.returncode}: {' '.join(cmd[-3:])}")
    warn = "\n".join(l for l in (res.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip())
    if verbose and warn:
        print(warn)


def build(verbose=False):
    objdir = os.path.join(os.path.dirname(HERE), "_build", "fdas")
    os.makedirs(objdir, exist_ok=True)
    inc = ["-I", os.path.join(os.path.dirname(HERE), "include")]
    jobs = []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        jobs.append(([hipcc()] + COMMON + inc + ["-c", src, "-o", obj], obj))
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(lambda j: _run(j[0], verbose), jobs))
    out_tmp = LIB + ".tmp"
    _run([hipcc()] + COMMON + ["-shared", "-o", out_tmp] + [o for _, o in jobs], verbose)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
