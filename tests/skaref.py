"""The FP64 oracle of the SKA-sized workload (2^22 bins, 16 pulsars, seed 2),
computed once per test process and shared by the test modules that compare
whole planes and whole candidate lists with it (test infrastructure; the
oracle is called, nothing of the library is).
"""

import functools
import os

import numpy as np

from oracle import fop as ofop
from oracle import harmonic as oh
from paper_1806_01556_amd import synth


def cpu_workers():
    """Threads this process may use: the scheduler's CPU set, or fewer when
    OMP_NUM_THREADS says so (it names the CPU share of a shared machine)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


@functools.lru_cache(maxsize=1)
def ska():
    """(spectrum complex64[2^22], pulsars, FOP float64[85][2^22], candidates, guard cells,
    per-plane population of the band |HP_k - T_k| <= 1e-2 T_k)."""
    spec, pulsars = synth.ska()
    print(f"oracle: FP64 FOP of the 2^22 workload on {cpu_workers()} threads", flush=True)
    plane64 = ofop.fop(spec.astype(np.complex128), workers=cpu_workers())
    print("oracle: harmonic sums of the 2^22 workload", flush=True)
    cands, guard, wide = oh.candidates_and_guard(plane64, 8, wide=WIDE)
    return spec, pulsars, plane64, cands, guard, wide


WIDE = 1e-2  # relative half-width of the band whose population gives the density at the thresholds


def assert_plane_close(got, ref, tol=1e-4, rows_per_step=8):
    """|got - ref| <= tol * max(ref, 1) for every cell of a (rows, n) plane;
    got may be wider than ref (columns past n are ignored).  Returns the worst
    |err| / bound."""
    worst = 0.0
    n = ref.shape[1]
    for r0 in range(0, ref.shape[0], rows_per_step):
        g = got[r0:r0 + rows_per_step, :n].astype(np.float64)
        f = ref[r0:r0 + rows_per_step]
        ratio = np.abs(g - f) / (tol * np.maximum(f, 1.0))
        m = float(np.max(ratio))
        if not m <= 1.0:  # also catches NaN
            bad = np.argwhere(~(ratio <= 1.0))
            raise AssertionError(f"{bad.shape[0]} cells off in rows {r0}..; first {bad[:5].tolist()}, worst {m:.3g}")
        worst = max(worst, m)
    return worst


def expected_guard_count(n, rows=85, n_harm=8, p_fa=1e-6, rel=1e-4):
    """Mean number of noise cells within rel*T_k of T_k, summed over the
    planes: rows * n * pdf_Gamma(k,1)(T_k) * 2 rel T_k (the band is thin)."""
    from scipy.stats import gamma
    t = oh.thresholds(n_harm, p_fa)
    return float(sum(rows * n * gamma.pdf(t[k - 1], k) * 2 * rel * t[k - 1] for k in range(1, n_harm + 1)))
