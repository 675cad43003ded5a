"""Pins for the oracle's harmonic summing, thresholds and candidates.

Independent anchors: hand-derived cells of the stretch map on a one-hot
plane, exact sums on constant planes, a pure-Python transcription of the loop
structure of Algorithm 1 on a tiny plane, the Erlang closed form for the
thresholds, and false-alarm counts on synthetic exponential noise.
"""

import numpy as np
import pytest

from oracle import harmonic


def erlang_survival(k, t):
    """P(Gamma(k,1) > t) = exp(-t) * sum_{n<k} t^n / n! (closed form, integer k)."""
    term, acc = 1.0, 1.0
    for n in range(1, k):
        term *= t / n
        acc += term
    return np.exp(-t) * acc


def test_thresholds_meet_false_alarm_probability():
    t = harmonic.thresholds(8, 1e-6)
    assert abs(t[0] - np.log(1e6)) < 1e-12
    for k in range(1, 9):
        assert abs(erlang_survival(k, t[k - 1]) / 1e-6 - 1.0) < 1e-9
    assert np.all(np.diff(t) > 0)


def _one_hot(z0, j0, z_max=4, n=40):
    p = np.zeros((2 * z_max + 1, n))
    p[z0 + z_max, j0] = 1.0
    return p


def _cells(plane, z_max=4):
    r, c = np.nonzero(plane)
    return sorted((int(a) - z_max, int(b)) for a, b in zip(r, c))


def test_stretch_cells_hand_derived_positive_row():
    # Source cell (i0, j0) = (3, 10).  HP_2 picks it up at (3, 10) [k=1] and
    # wherever trunc(i/2) = 3 and floor(j/2) = 10: i in {6, 7}, j in {20, 21}.
    # z_max = 8 so rows 6, 7 exist.
    p = _one_hot(3, 10, z_max=8, n=40)
    planes = dict(harmonic.harmonic_planes(p, 3))
    assert _cells(planes[1], 8) == [(3, 10)]
    assert _cells(planes[2], 8) == [(3, 10), (6, 20), (6, 21), (7, 20), (7, 21)]
    # k=3 adds trunc(i/3) = 3 -> i in {9, 10, 11} (outside z_max = 8) -> nothing new
    assert _cells(planes[3], 8) == _cells(planes[2], 8)


def test_stretch_cells_hand_derived_negative_and_zero_rows():
    # trunc toward zero: trunc(i/2) = -1 for i in {-2, -3}; floor(j/2) = 5 for j in {10, 11}.
    p = _one_hot(-1, 5, z_max=4, n=16)
    hp2 = dict(harmonic.harmonic_planes(p, 2))[2]
    assert _cells(hp2, 4) == [(-3, 10), (-3, 11), (-2, 10), (-2, 11), (-1, 5)]
    # row 0 is the source of rows -1, 0, 1 for k = 2, and of -2..2 for k = 3.
    p = _one_hot(0, 2, z_max=4, n=12)
    hp3 = dict(harmonic.harmonic_planes(p, 3))[3]
    expect = {(0, 2): 1.0}
    for i in (-1, 0, 1):
        for j in (4, 5):
            expect[(i, j)] = expect.get((i, j), 0.0) + 1.0
    for i in (-2, -1, 0, 1, 2):
        for j in (6, 7, 8):
            expect[(i, j)] = expect.get((i, j), 0.0) + 1.0
    got = {(int(r) - 4, int(c)): hp3[r, c] for r, c in zip(*np.nonzero(hp3))}
    assert got == expect


def test_constant_plane_sums_to_k_times_value():
    p = np.full((85, 257), 0.75)
    for k, hp in harmonic.harmonic_planes(p, 8):
        assert np.all(hp == 0.75 * k)


def test_first_plane_is_fop_and_planes_increase():
    rng = np.random.default_rng(4)
    p = rng.exponential(size=(85, 1000)).astype(np.float32)
    prev = None
    for k, hp in harmonic.harmonic_planes(p, 8):
        if k == 1:
            assert np.array_equal(hp, p)
        else:
            assert np.all(hp >= prev)
        prev = hp


def test_vectorised_planes_match_algorithm1_loops():
    # Literal loop structure of Algorithm 1 on a tiny plane (pure Python).
    rng = np.random.default_rng(7)
    z_max, n, nh = 3, 30, 5
    fop = rng.random((2 * z_max + 1, n))
    hp_prev = [[0.0] * n for _ in range(2 * z_max + 1)]
    loops = {}
    for k in range(1, nh + 1):
        hp = [[0.0] * n for _ in range(2 * z_max + 1)]
        for i in range(-z_max, z_max + 1):
            for j in range(n):
                si = int(i / k)  # C-style truncation
                sp = fop[si + z_max][j // k]
                hp[i + z_max][j] = hp_prev[i + z_max][j] + sp
        loops[k] = np.array(hp)
        hp_prev = hp
    for k, hp in harmonic.harmonic_planes(fop, nh):
        assert np.array_equal(hp, loops[k])


def test_false_alarm_rate_on_exponential_noise():
    # FOP cells of pure noise are Exp(1); for columns j >= 56 the k source
    # cells of HP_k are distinct, so HP_k ~ Gamma(k) and the count above
    # T_k(p_fa) is Binomial(cells, p_fa).
    rng = np.random.default_rng(12)
    p_fa = 2e-3
    plane = rng.exponential(size=(85, 24000))
    t = harmonic.thresholds(8, p_fa)
    for k, hp in harmonic.harmonic_planes(plane, 8):
        sub = hp[:, 56:]
        cnt = int(np.count_nonzero(sub > t[k - 1]))
        mu = sub.size * p_fa
        # HP_k cells share sources, so counts are positively correlated; allow 8 sigma
        assert abs(cnt - mu) < 8 * np.sqrt(mu * k), (k, cnt, mu)


def test_candidates_order_counts_and_topk():
    rng = np.random.default_rng(3)
    plane = rng.exponential(size=(85, 5000)) * 3.0
    c = harmonic.candidates(plane, 8)
    key = list(zip(c["harm"], c["z"], c["r"]))
    assert key == sorted(key)
    for rec in c[:50]:
        k, z, r = int(rec["harm"]), int(rec["z"]), int(rec["r"])
        hp = dict(harmonic.harmonic_planes(plane, k))[k]
        assert hp[z + 42, r] == rec["power"]
        assert rec["power"] > harmonic.thresholds(8)[k - 1]
    top = harmonic.candidates(plane, 8, top_k=200)
    counts = harmonic.plane_counts(top)
    full = harmonic.plane_counts(c)
    assert np.all(counts == np.minimum(full, 200))
    for k in range(1, 9):
        sel_full = np.sort(c["power"][c["harm"] == k])[::-1]
        sel_top = np.sort(top["power"][top["harm"] == k])[::-1]
        assert np.array_equal(sel_top, sel_full[:200])


def test_fp32_twin_sums_in_k_order():
    # FP32 plane: every step is one float32 rounding of (HP_{k-1} + SP_k).
    rng = np.random.default_rng(9)
    p = (rng.exponential(size=(85, 777)) * 7).astype(np.float32)
    acc = p.copy()
    for k, hp in harmonic.harmonic_planes(p, 8):
        assert hp.dtype == np.float32
        if k > 1:
            rows = harmonic.stretch_rows(k)
            cols = harmonic.stretch_cols(k, p.shape[1])
            acc = (acc + p[rows][:, cols]).astype(np.float32)
        assert np.array_equal(hp, acc)


def test_column_window_equals_restriction_of_full_plane():
    rng = np.random.default_rng(1)
    p = rng.exponential(size=(85, 6000)) * 3
    full = harmonic.candidates(p, 8)
    w = np.arange(2000, 3500)
    win = harmonic.candidates(p, 8, cols=w)
    sel = full[(full["r"] >= 2000) & (full["r"] < 3500)]
    assert win.size > 1000 and np.array_equal(sel, win)


def _guard_pin_plane(ta, n=4000):
    """A 2*4+1-row plane of zeros whose harmonic sums sit at chosen distances
    from the thresholds.  Every set cell has column j >= n/2, so the stretched
    sources floor(j/k) < n/2 of every plane k >= 2 are zero and HP_k(i, j) is
    the cell's own value for every k, except the last group, which also sets
    the source floor(j/2) so that only HP_2 (and higher) carries the sum."""
    z_max, rows = 4, 9
    p = np.zeros((rows, n))
    placed = []  # (k, z, r, value, expected in the band of plane k)
    j = n // 2
    for k in range(1, ta.shape[0] + 1):
        for z in (-4, -1, 0, 3):
            t = ta[k - 1, z + z_max]
            for f, inside in ((1 + 0.5e-4, True), (1 - 0.5e-4, True), (1 + 2e-4, False), (1 - 2e-4, False)):
                p[z + z_max, j] = t * f
                placed.append((k, z, j, t * f, inside))
                j += 3
    # HP_2 = a + b with a at (z, j) and b at its k = 2 source (trunc(z/2), floor(j/2))
    extra = []
    for z in (2, -3):
        jj = j + (j % 2)
        a = 1.0
        b = ta[1, z + z_max] * (1 + 0.3e-4) - a
        p[z + z_max, jj] = a
        p[int(np.trunc(z / 2)) + z_max, jj // 2] = b
        extra.append((z, jj))
        j = jj + 4
    assert j < n
    return p, placed, extra


@pytest.mark.parametrize("row_dependent", [False, True])
def test_guard_cells_band_width_and_plane(row_dependent):
    """guard_cells keeps exactly the cells whose FP64 HP_k is within 1e-4 T of
    plane k's own threshold TA(k, i): 0.5e-4 T away is in, 2e-4 T is out, for
    every k, for negative, zero and positive rows, and for a threshold that
    depends on the row; a sum of two cells is judged on HP_2, not on the FOP."""
    ta = harmonic.threshold_array(8, 4, 1e-6)
    if row_dependent:
        ta = ta * (1.0 + 0.03 * np.arange(9)[None, :])
    p, placed, extra = _guard_pin_plane(ta)
    guard = harmonic.guard_cells(p, 8, ta=ta)
    for k, z, r, v, inside in placed:
        assert ((k, z, r) in guard) == inside, (k, z, r, v / ta[k - 1, z + 4])
        # the value is never within the band of another plane's threshold
        for k2 in range(1, 9):
            if k2 != k:
                assert (k2, z, r) not in guard
    for z, jj in extra:
        assert (2, z, jj) in guard and (1, z, jj) not in guard
    # one pass gives the same list and band
    c1 = harmonic.candidates(p, 8, ta=ta)
    c2, g2 = harmonic.candidates_and_guard(p, 8, ta=ta)
    assert g2 == guard
    assert np.array_equal(c1, c2)
    # the cells just above threshold are candidates of their plane
    keys = set(zip(c1["harm"].tolist(), c1["z"].tolist(), c1["r"].tolist()))
    for k, z, r, v, inside in placed:
        if v > ta[k - 1, z + 4]:
            assert (k, z, r) in keys


def test_candidates_and_guard_one_pass_matches_on_noise():
    rng = np.random.default_rng(44)
    plane = rng.exponential(size=(85, 30000))
    ta = harmonic.threshold_array(8, 42, 1e-3)
    c, g = harmonic.candidates_and_guard(plane, 8, ta=ta, rel=1e-2)
    assert np.array_equal(c, harmonic.candidates(plane, 8, ta=ta))
    assert g == harmonic.guard_cells(plane, 8, ta=ta, rel=1e-2)
    assert len(g) > 50
    cols = np.arange(1000, 9000)
    c, g = harmonic.candidates_and_guard(plane, 8, ta=ta, rel=1e-2, cols=cols)
    assert np.array_equal(c, harmonic.candidates(plane, 8, ta=ta, cols=cols))
    assert g == harmonic.guard_cells(plane, 8, ta=ta, rel=1e-2, cols=cols)


def test_guard_count_on_noise_matches_the_band_density():
    """On exponential noise the band holds about rows * n * f_k(T_k) * 2 rel T_k
    cells per plane (a wide band, rel = 0.02, so the count is large), and
    about rel / wide of the cells of a band `wide` times as wide."""
    rng = np.random.default_rng(45)
    n = 200000
    plane = rng.exponential(size=(85, n))
    _, g, w = harmonic.candidates_and_guard(plane, 1, p_fa=1e-3, rel=0.02, wide=0.2)
    from skaref import expected_guard_count
    mean = expected_guard_count(n, n_harm=1, p_fa=1e-3, rel=0.02)
    assert abs(len(g) - mean) <= 5 * np.sqrt(mean), (len(g), mean)
    # the density is not flat over +-20 %: Gamma(1) falls by e^{+-0.2 T}; the
    # band population of the exponential is exact, 2 sinh(0.2 T) e^{-T} per cell
    T = harmonic.thresholds(1, 1e-3)[0]
    wide_mean = 85 * n * 2 * np.sinh(0.2 * T) * np.exp(-T)
    assert abs(w[0] - wide_mean) <= 5 * np.sqrt(wide_mean), (w[0], wide_mean)
