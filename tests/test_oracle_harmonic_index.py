"""Pins of the oracle's alternative harmonic index maps (CPU).

"fundamental": HP_k(i, j) = HP_{k-1}(i, j) + FOP(k i, k j), 0 outside the plane.
"highest":     HP_k(i, j) = sum_{m<=k} FOP(rho(m i, k), rho(m j, k)).

Both are pinned by what harmonically related signals fix, not by retyping the
formulas: planted harmonic spikes are collected exactly at the anchor cell,
constant planes give term counts, the two maps agree where the highest-anchored
map samples exact multiples, and an injected pulsar with integer (r, z) is
recovered at the predicted cells through the whole oracle pipeline.
"""

import numpy as np
import pytest

from oracle import fop as ofop
from oracle import harmonic as oh
from paper_1806_01556_amd import synth

Z, N = 42, 4000


def _spikes(z0, r0, amps):
    """A zero plane with value amps[m-1] at (m z0, m r0), m = 1.."""
    plane = np.zeros((2 * Z + 1, N))
    for m, a in enumerate(amps, start=1):
        plane[m * z0 + Z, m * r0] = a
    return plane


def test_fundamental_collects_harmonics_at_the_fundamental():
    amps = [1000.0, 100.0, 10.0, 1.0]  # falling with m, as a pulsar's harmonics
    plane = _spikes(7, 300, amps)
    for k, hp in oh.harmonic_planes(plane, 4, index="fundamental"):
        assert hp[7 + Z, 300] == sum(amps[:k])
        # the anchor is the only cell that sees every harmonic: the unique maximum
        other = hp.copy()
        other[7 + Z, 300] = 0.0
        assert other.max() < hp[7 + Z, 300]


def test_highest_collects_harmonics_at_the_highest():
    amps = [1.0, 10.0, 100.0, 1000.0]
    plane = _spikes(5, 200, amps)
    for k, hp in oh.harmonic_planes(plane, 4, index="highest"):
        assert hp[k * 5 + Z, k * 200] == sum(amps[:k])


def test_first_plane_is_the_fop():
    plane = np.random.default_rng(3).exponential(size=(2 * Z + 1, 300))
    for index in ("fundamental", "highest", "stretch"):
        k, hp = next(oh.harmonic_planes(plane, 1, index=index))
        assert k == 1 and np.array_equal(hp, plane)


def test_constant_plane_counts_terms():
    n = 500
    plane = np.ones((2 * Z + 1, n))
    i = np.arange(-Z, Z + 1)[:, None]
    j = np.arange(n)[None, :]
    for k, hp in oh.harmonic_planes(plane, 8, index="fundamental"):
        terms = sum(((np.abs(m * i) <= Z) & (m * j < n)).astype(float) for m in range(1, k + 1))
        assert np.array_equal(hp, terms)
    for k, hp in oh.harmonic_planes(plane, 8, index="highest"):
        assert np.all(hp == k)  # every term is inside the plane


def test_rounding_is_half_away_from_zero():
    assert list(oh.round_half_away([-7, -5, -3, -1, 0, 1, 3, 5, 7], 2)) == [-4, -3, -2, -1, 0, 1, 2, 3, 4]
    assert list(oh.round_half_away([1, 2, 4, 5, 7, 8], 3)) == [0, 1, 1, 2, 2, 3]


def test_highest_equals_fundamental_on_exact_multiples():
    # at (k i, k j) the highest-anchored plane k samples (m i, m j) exactly,
    # which is what the fundamental-anchored plane k sums at (i, j)
    rng = np.random.default_rng(11)
    plane = rng.exponential(size=(2 * Z + 1, N))
    fund = dict(oh.harmonic_planes(plane, 6, index="fundamental"))
    high = dict(oh.harmonic_planes(plane, 6, index="highest"))
    for k in range(1, 7):
        for i in range(-(Z // k), Z // k + 1):
            js = np.arange(0, (N - 1) // k + 1, 37)
            np.testing.assert_allclose(high[k][k * i + Z, k * js], fund[k][i + Z, js], rtol=1e-12)


def test_injected_pulsar_recovered_by_both_maps():
    # integer (r, z): the matched template peaks exactly on the cell
    r0, z0, snr = 12000, 10, 12.0  # harmonics 2..4 at (24000, 20) .. (48000, 40), all inside 2^16 bins
    spec, _ = synth.make_spectrum(1 << 16, 21, pulsars=[synth.Pulsar(r=float(r0), z=float(z0), snr=snr, n_harm=4)])
    plane = ofop.fop(spec.astype(np.complex128))
    fund = oh.candidates(plane, 4, index="fundamental")
    high = oh.candidates(plane, 4, index="highest")
    fk = set(zip(fund["harm"].tolist(), fund["z"].tolist(), fund["r"].tolist()))
    hk = set(zip(high["harm"].tolist(), high["z"].tolist(), high["r"].tolist()))
    for k in range(1, 5):
        assert (k, z0, r0) in fk
        assert (k, k * z0, k * r0) in hk
    # each harmonic adds about (snr/m)^2 at the fundamental-anchored cell
    hp = dict(oh.harmonic_planes(plane, 4, index="fundamental"))
    steps = [hp[k][z0 + Z, r0] - (hp[k - 1][z0 + Z, r0] if k > 1 else 0.0) for k in range(1, 5)]
    expect = [(snr / m) ** 2 for m in range(1, 5)]
    for got, ref in zip(steps, expect):
        assert abs(got - ref) < 4.0 * np.sqrt(ref) + 3.0


def test_unknown_index_rejected():
    with pytest.raises(ValueError):
        next(oh.harmonic_planes(np.zeros((3, 4)), 2, index="nope"))
