"""Pins for the oracle's acceleration response and templates.

Each check compares the oracle with something it does not compute itself:
the defining integral by independent quadrature (numpy Gauss-Legendre and
mpmath), the elementary z = 0 case, Parseval's theorem, and the DFT of a
sampled chirp made by the input generator.
"""

import json
import os

import numpy as np
import pytest

from oracle import response

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def quad_response(q, z, panels=1024, order=16):
    """integral_0^1 exp(i*pi*(z u^2 + (2q - z) u)) du by composite Gauss-Legendre."""
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 1.0, panels + 1)
    a, b = edges[:-1], edges[1:]
    u = (0.5 * (b - a))[:, None] * x[None, :] + (0.5 * (a + b))[:, None]
    wu = (0.5 * (b - a))[:, None] * w[None, :]
    u = u.ravel()
    wu = wu.ravel()
    q = np.atleast_1d(np.asarray(q, dtype=np.float64))
    ph = np.pi * (z * u[None, :] ** 2 + (2.0 * q[:, None] - z) * u[None, :])
    return (np.exp(1j * ph) * wu[None, :]).sum(axis=1)


def test_tap_counts_match_rule_and_bound():
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_table1.json")) as f:
        t1 = json.load(f)
    zs = range(-42, 43)
    L = [response.tap_count(z) for z in zs]
    assert len(L) == t1["N_temp"]
    assert L[42] == 16 and response.tap_count(1) == 26 and response.tap_count(-42) == 394
    assert max(L) <= t1["N_tap_bound_section1"]
    assert sum(L) == 17656
    for z in zs:
        d = response.tap_offsets(z)
        assert d[0] == -response.tap_count(z) // 2 and d[-1] == response.tap_count(z) // 2 - 1


def test_z0_response_is_delta_at_integer_offsets():
    q = np.arange(-300, 301)
    a = response.response(q, 0)
    assert abs(a[300] - 1.0) < 1e-15
    off = np.delete(a, 300)
    assert np.max(np.abs(off)) < 1e-15
    d, h = response.template(0)
    expect = (d == 0).astype(np.complex128)
    assert np.max(np.abs(h - expect)) < 1e-15


@pytest.mark.parametrize("z", [1, 2, 3, 5, 17, 42, -1, -4, -29, -42])
def test_closed_form_matches_gauss_legendre_quadrature(z):
    q = np.arange(-260, 261)
    a = response.response(q, z)
    ref = quad_response(q, z)
    assert np.max(np.abs(a - ref)) < 1e-12


def test_closed_form_matches_mpmath_quadrature():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 30
    for z, q in [(1, 0), (1, 37), (7, -3), (17, 9), (42, -150), (-23, 41), (-42, 197)]:
        f = lambda u: mpmath.expj(mpmath.pi * (z * u * u + (2 * q - z) * u))
        pts = mpmath.linspace(0, 1, 80)
        ref = complex(mpmath.quad(f, pts))
        got = complex(response.response(np.array([q]), z)[0])
        assert abs(got - ref) < 1e-13, (z, q, got, ref)


@pytest.mark.parametrize("z", [0, 1, 6, 21, 42, -13])
def test_parseval_sum_over_integer_offsets_is_one(z):
    # sum_q |A(q,z)|^2 = integral_0^1 |exp(i pi z (u^2 - u))|^2 du = 1 (Parseval);
    # the tail beyond |q| = Q is about 1/(pi^2 Q).
    Q = 400000
    q = np.arange(-Q, Q + 1)
    s = np.sum(np.abs(response.response(q, z)) ** 2)
    assert abs(s - 1.0) < 3.0 / (np.pi ** 2 * Q)


@pytest.mark.parametrize("z", [0, 3, 17, 42, -42])
def test_templates_have_unit_energy_and_near_full_support(z):
    d, h = response.template(z)
    assert abs(np.sum(np.abs(h) ** 2) - 1.0) < 1e-13
    assert response.support_energy(z) > 0.9999


def test_sampled_chirp_dft_matches_response():
    # A chirp made by the input generator (time domain, FP64 DFT) must land on
    # A(r_c - k, z) up to the discretisation error of sampling u = n/N.
    from paper_1806_01556_amd import synth

    n = 8192
    for r_c, z in [(1000.0, 0.0), (2000.0, 12.0), (3000.0, -33.0), (1500.0, 42.0)]:
        x = synth._chirp_series(n, r_c, z, 1.0, 0.0)
        X = np.fft.fft(x)
        k = np.arange(int(r_c) - 300, int(r_c) + 301)
        a = response.response(int(r_c) - k, int(z))
        assert np.max(np.abs(X[k] - a)) < 1e-6, (r_c, z)

