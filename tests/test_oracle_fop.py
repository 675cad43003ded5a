"""Pins for the oracle's FT convolution (filter-output plane).

Independent anchors: a pure-Python double loop of eq. (1) on tiny inputs, the
z = 0 template reducing the row to |X|^2, the matched-filter peak of a
noise-free signal built by separate quadrature, linearity/shift properties,
the unit mean of noise power, and recovery of a chirp injected by the input
generator at its known (r, z).
"""

import numpy as np
import pytest

from oracle import fop, response
from paper_1806_01556_amd import synth


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_direct_sum_matches_python_double_loop():
    x = _rand(48, 11)
    for z in [0, 2, -3]:
        d, h = response.template(z)
        y = fop.correlate_direct(x, d, h)
        for j in range(x.size):
            acc = 0j
            for dd, hh in zip(d, h):
                if 0 <= j + dd < x.size:
                    acc += x[j + dd] * hh
            assert abs(y[j] - acc) < 1e-12


@pytest.mark.parametrize("n", [1, 7, 400, 1000, 4096])
def test_fft_form_equals_direct_sum(n):
    # eq. (1) and eq. (2) give the same filter output.
    x = _rand(n, n)
    a = fop.fop(x, z_max=42, method="fft")
    b = fop.fop(x, z_max=42, method="direct")
    assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(b))


def test_z0_row_is_bin_power():
    x = _rand(5000, 3)
    plane = fop.fop(x)
    assert np.max(np.abs(plane[42] - np.abs(x) ** 2)) < 1e-12 * np.max(np.abs(x) ** 2)


@pytest.mark.parametrize("z0", [-37, -5, 0, 9, 42])
def test_matched_filter_peak_at_true_cell(z0):
    # Noise-free X[k] = a * A(r - k, z0) with A from an independent quadrature:
    # the correlation at (z0, r) is a * sqrt(E_z0), so FOP = a^2 * E_z0, and it
    # is the largest value of the plane.
    from test_oracle_response import quad_response

    n, r, a = 3000, 1500, 3.0
    k = np.arange(n)
    x = a * quad_response(r - k, z0, panels=512)
    plane = fop.fop(x)
    e = response.support_energy(z0)
    assert abs(plane[z0 + 42, r] - a * a * e) < 1e-9 * a * a
    row, col = np.unravel_index(np.argmax(plane), plane.shape)
    assert (row - 42, col) == (z0, r)


def test_linearity_and_shift():
    n = 3000
    x1, x2 = _rand(n, 5), _rand(n, 6)
    d, h = response.template(11)
    y1 = fop.correlate_fft(x1, d, h)
    y2 = fop.correlate_fft(x2, d, h)
    y12 = fop.correlate_fft(2.0 * x1 - 0.5j * x2, d, h)
    assert np.max(np.abs(y12 - (2.0 * y1 - 0.5j * y2))) < 1e-10
    s = 37
    xs = np.zeros(n, dtype=np.complex128)
    xs[s:] = x1[:-s]
    ys = fop.correlate_fft(xs, d, h)
    lo, hi = s + 200, n - 200
    assert np.max(np.abs(ys[lo:hi] - y1[lo - s:hi - s])) < 1e-10


def test_noise_power_has_unit_mean_in_every_row():
    # Unit-variance complex noise through unit-energy templates: power ~ Exp(1).
    n = 1 << 15
    x = synth.noise_only(n, 99).astype(np.complex128)
    plane = fop.fop(x)
    m = plane[:, 256:-256].mean(axis=1)
    # standard error of a mean of ~3e4 correlated-within-a-template-width samples
    assert np.all(np.abs(m - 1.0) < 0.05), m


def test_injected_pulsar_recovered_at_known_cell():
    # The small workload's pulsar: r = 20000.3, z = 17.5, SNR 10, noise free.
    n = 1 << 16
    spec = np.zeros(n, dtype=np.complex128)
    p = synth.Pulsar(r=20000.3, z=17.5, snr=10.0, n_harm=1)
    synth.inject(spec, [p], np.random.default_rng(0))
    plane = fop.fop(spec)
    row, col = np.unravel_index(np.argmax(plane), plane.shape)
    assert row - 42 in (17, 18) and col in (20000, 20001)
    # scalloping from half-bin offsets in r and z keeps the peak below SNR^2
    assert 0.4 * 100 < plane[row, col] < 100


def test_points_match_full_plane():
    x = _rand(2000, 8)
    plane = fop.fop(x)
    rng = np.random.default_rng(1)
    rows = rng.integers(0, 85, 300)
    cols = rng.integers(0, 2000, 300)
    pts = fop.fop_points(x, rows, cols)
    assert np.max(np.abs(pts - plane[rows, cols])) < 1e-10 * max(1.0, plane.max())
