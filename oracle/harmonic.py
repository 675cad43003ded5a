"""Harmonic summing, thresholds and candidates (oracle, FP64 plus an FP32 twin).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

Algorithm 1 (Section 2.2): the FOP is stretched by the integers k = 1..N_hp
into stretch planes SP_k, the harmonic planes accumulate them,
HP_k = HP_{k-1} + SP_k (HP_0 = 0, so HP_1 = FOP), and threshold detection
against TA(k, i) collects candidates from every plane.  N_hp = 8 and
N_cand = 200 (Table 1).

Readings (the paper defines neither ``stretch`` nor TA):

* stretch: SP_k(i, j) = FOP(trunc(i / k), floor(j / k)), i the signed row
  index -(N_temp-1)/2..(N_temp-1)/2, j the column.  Integer division, C
  semantics for the signed row (truncation toward zero), so every source index
  lies inside the plane for every (i, j, k), as the full loops of Algorithm 1
  require.
* TA(k, i) = T_k, the power at which a sum of k independent unit-mean
  exponential powers (Gamma(k, 1), the noise law of HP_k for unit-energy
  templates and unit-variance complex noise) exceeds with probability p_fa:
  T_k = Q^{-1}(k, p_fa), Q the regularised upper incomplete gamma function.
  The default p_fa is 1e-6 per cell.
* detection: strict HP_k(i, j) > TA(k, i); a candidate is (k, i, j, HP_k).

Two further index maps (alternatives to the stretch reading, selected with
``index``), both written from the physics of harmonically related signals: a
pulsar whose fundamental sits at (z, r) has its m-th harmonic at (m z, m r).

* "fundamental": plane k is anchored on the fundamental,
  HP_k(i, j) = HP_{k-1}(i, j) + FOP(k i, k j), a term being 0 where (k i, k j)
  lies outside the plane (|k i| > z_max or k j >= N).  Cumulative in k like
  Algorithm 1.
* "highest": plane k is anchored on the k-th (highest) harmonic,
  HP_k(i, j) = sum_{m=1..k} FOP(rho(m i, k), rho(m j, k)), summed in m order,
  rho(a, k) = a / k rounded to the nearest integer, halves away from zero.
  Every index lies inside the plane; the planes are not cumulative.
  The list is given in (k, i, j) order, the loop order of Algorithm 1.
  Keeping only N_cand per plane is optional ("top_k"): the highest powers,
  ties broken by (i, j) ascending.
"""

import numpy as np
from scipy.special import gammainccinv

CAND_DTYPE = np.dtype([("harm", np.int32), ("z", np.int32), ("r", np.int32), ("power", np.float64)])


def stretch_rows(k, z_max=42):
    """Row (0-based, row = i + z_max) that SP_k reads for every output row."""
    i = np.arange(-z_max, z_max + 1, dtype=np.int64)
    src = np.sign(i) * (np.abs(i) // k)  # trunc(i / k)
    return src + z_max


def stretch_cols(k, n, cols=None):
    """Column that SP_k reads for every output column: floor(j / k).

    ``cols`` restricts the output columns (default: all n)."""
    j = np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    return j // k


def stretch_plane(plane, k, cols=None):
    """SP_k of Algorithm 1 (reading above): a gathered copy of the plane.

    ``cols`` evaluates only those output columns (same definition)."""
    z_max = (plane.shape[0] - 1) // 2
    rows = stretch_rows(k, z_max)
    src = stretch_cols(k, plane.shape[1], cols)
    return plane[np.ix_(rows, src)]


def harmonic_planes(plane, n_harm=8, cols=None, index="stretch"):
    """Yield (k, HP_k) for k = 1..n_harm in the plane's own dtype.

    The sum is formed in k order, one rounding per step, exactly as
    HP_k = HP_{k-1} + SP_k; with a float32 plane this is the FP32 twin that a
    GPU kernel summing in the same order must reproduce bit for bit.
    ``cols`` evaluates only those output columns.  ``index`` selects the
    index map: "stretch" (Algorithm 1 with the reading above), "fundamental"
    or "highest" (see the module notes).
    """
    if index == "fundamental":
        yield from _planes_fundamental(plane, n_harm, cols)
        return
    if index == "highest":
        yield from _planes_highest(plane, n_harm, cols)
        return
    if index != "stretch":
        raise ValueError(f"unknown index map {index!r}")
    ncols = plane.shape[1] if cols is None else len(cols)
    hp = np.zeros((plane.shape[0], ncols), dtype=plane.dtype)
    for k in range(1, n_harm + 1):
        hp = hp + stretch_plane(plane, k, cols)
        yield k, hp


def _planes_fundamental(plane, n_harm, cols):
    """HP_k = HP_{k-1} + FOP(k i, k j), zero outside the plane."""
    rows, n = plane.shape
    z_max = (rows - 1) // 2
    j = np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    i = np.arange(-z_max, z_max + 1, dtype=np.int64)
    hp = np.zeros((rows, j.size), dtype=plane.dtype)
    for k in range(1, n_harm + 1):
        si, sj = k * i, k * j
        ri, rj = np.abs(si) <= z_max, sj < n
        sp = np.zeros_like(hp)
        sp[np.ix_(ri, rj)] = plane[np.ix_(si[ri] + z_max, sj[rj])]
        hp = hp + sp
        yield k, hp


def round_half_away(a, k):
    """a / k rounded to the nearest integer, halves away from zero (integers)."""
    a = np.asarray(a, dtype=np.int64)
    return np.sign(a) * ((2 * np.abs(a) + k) // (2 * k))


def _planes_highest(plane, n_harm, cols):
    """HP_k = sum_{m=1..k} FOP(rho(m i, k), rho(m j, k)), in m order."""
    rows, n = plane.shape
    z_max = (rows - 1) // 2
    j = np.arange(n, dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    i = np.arange(-z_max, z_max + 1, dtype=np.int64)
    for k in range(1, n_harm + 1):
        hp = np.zeros((rows, j.size), dtype=plane.dtype)
        for m in range(1, k + 1):
            hp = hp + plane[np.ix_(round_half_away(m * i, k) + z_max, round_half_away(m * j, k))]
        yield k, hp


def thresholds(n_harm=8, p_fa=1e-6):
    """T_k = Q^{-1}(k, p_fa), k = 1..n_harm (FP64)."""
    return np.array([gammainccinv(k, p_fa) for k in range(1, n_harm + 1)], dtype=np.float64)


def threshold_array(n_harm=8, z_max=42, p_fa=1e-6):
    """TA(k, i) as an (n_harm, 2*z_max+1) array, row-independent."""
    t = thresholds(n_harm, p_fa)
    return np.repeat(t[:, None], 2 * z_max + 1, axis=1)


def candidates(plane, n_harm=8, ta=None, p_fa=1e-6, top_k=0, cols=None, index="stretch"):
    """Candidate list of Algorithm 1 as a CAND_DTYPE array in (k, i, j) order.

    plane: FOP (rows = templates, columns = bins), float64 or float32.  With a
    float32 plane the sums and the comparisons are done in float32 (TA rounded
    to float32), which is the arithmetic of the GPU kernel.  ``cols`` (an
    increasing array of output columns) restricts detection to those columns.
    """
    colidx = np.arange(plane.shape[1], dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    z_max = (plane.shape[0] - 1) // 2
    if ta is None:
        ta = threshold_array(n_harm, z_max, p_fa)
    ta = np.asarray(ta, dtype=plane.dtype)
    out = []
    for k, hp in harmonic_planes(plane, n_harm, cols, index):
        rows, cc = np.nonzero(hp > ta[k - 1][:, None])
        cols_k = colidx[cc]
        pw = hp[rows, cc].astype(np.float64)
        if top_k and rows.size > top_k:
            # highest power first, ties by (i, j) ascending
            order = np.lexsort((cols_k, rows, -pw))[:top_k]
            rows, cols_k, pw = rows[order], cols_k[order], pw[order]
        rec = np.empty(rows.size, dtype=CAND_DTYPE)
        rec["harm"] = k
        rec["z"] = rows - z_max
        rec["r"] = cols_k
        rec["power"] = pw
        out.append(rec)
    allc = np.concatenate(out) if out else np.empty(0, dtype=CAND_DTYPE)
    order = np.lexsort((allc["r"], allc["z"], allc["harm"]))
    return allc[order]


def plane_counts(cands, n_harm=8):
    """Candidates per harmonic plane."""
    return np.bincount(cands["harm"] - 1, minlength=n_harm).astype(np.int64)


def guard_cells(plane, n_harm=8, ta=None, p_fa=1e-6, rel=1e-4, cols=None, index="stretch"):
    """Cells whose FP64 harmonic sum lies within rel*T of the threshold.

    Returned as a set of (k, z, r).  A correct FP32 implementation may report
    these either way, since its rounding can move them across the threshold.
    """
    z_max = (plane.shape[0] - 1) // 2
    if ta is None:
        ta = threshold_array(n_harm, z_max, p_fa)
    ta = np.asarray(ta, dtype=np.float64)
    colidx = np.arange(plane.shape[1], dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    out = set()
    for k, hp in harmonic_planes(np.asarray(plane, dtype=np.float64), n_harm, cols, index):
        t = ta[k - 1][:, None]
        rows, cc = np.nonzero(np.abs(hp - t) <= rel * t)
        out.update((k, int(r) - z_max, int(colidx[c])) for r, c in zip(rows, cc))
    return out


def candidates_and_guard(plane, n_harm=8, ta=None, p_fa=1e-6, rel=1e-4, cols=None, wide=None):
    """candidates(plane, ...) and guard_cells(plane, ...) of an FP64 plane in
    one pass over its harmonic planes (the same definitions, each plane
    formed once): (CAND_DTYPE array in (k, i, j) order, set of (k, z, r)).

    With ``wide`` a third element is returned: per plane, the number of cells
    with |HP_k - TA(k, i)| <= wide * TA(k, i), the population of a wider band
    from which the density of harmonic sums around the threshold is read."""
    plane = np.asarray(plane, dtype=np.float64)
    z_max = (plane.shape[0] - 1) // 2
    if ta is None:
        ta = threshold_array(n_harm, z_max, p_fa)
    ta = np.asarray(ta, dtype=np.float64)
    colidx = np.arange(plane.shape[1], dtype=np.int64) if cols is None else np.asarray(cols, dtype=np.int64)
    out, guard, wide_counts = [], set(), []
    for k, hp in harmonic_planes(plane, n_harm, cols):
        t = ta[k - 1][:, None]
        rows, cc = np.nonzero(hp > t)
        rec = np.empty(rows.size, dtype=CAND_DTYPE)
        rec["harm"] = k
        rec["z"] = rows - z_max
        rec["r"] = colidx[cc]
        rec["power"] = hp[rows, cc]
        out.append(rec)
        dist = np.abs(hp - t)
        grows, gcc = np.nonzero(dist <= rel * t)
        guard.update((k, int(r) - z_max, int(colidx[c])) for r, c in zip(grows, gcc))
        if wide is not None:
            wide_counts.append(int(np.count_nonzero(dist <= wide * t)))
    allc = np.concatenate(out) if out else np.empty(0, dtype=CAND_DTYPE)
    order = np.lexsort((allc["r"], allc["z"], allc["harm"]))
    if wide is None:
        return allc[order], guard
    return allc[order], guard, np.array(wide_counts, dtype=np.int64)
