"""Fourier-domain acceleration response and templates (oracle, FP64).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

The paper (Section 1 and Section 2) builds FDAS on the correlation technique of
Ransom et al.: each of the N_temp = 85 FIR filters (Table 1) is the complex
conjugate response of a signal whose frequency drifts linearly by z Fourier
bins over the observation.  The paper gives the filter count, the row range
of the filter-output plane (Algorithm 1: i = -(N_temp-1)/2 .. (N_temp-1)/2)
and the bound of about 400 taps (Section 1), but not the coefficients.
Readings used here:

* Response.  A signal with mean Fourier frequency r_c and total drift z bins,
  observed for u in [0, 1), has the (normalised) Fourier response at bin k

      A(q, z) = integral_0^1 exp(i*pi*(z*u^2 + (2q - z)*u)) du,  q = r_c - k.

* Template row i has z = i (unit step in z).
* Template z has L(z) = 2*(8 + ceil(4.5|z|)) taps at offsets
  d in [-L/2, L/2 - 1]; L(42) = 394 fits the ~400-tap bound of Section 1.
* h_z[d] = conj(A(-d, z)) / sqrt(E_z) with E_z = sum_d |A(-d, z)|^2 over the
  support, so each template has unit energy.

``response`` evaluates A in closed form.  Completing the square in the
exponent with p = q - z/2 gives, for z > 0,

      A = exp(-i*pi*p^2/z) / sqrt(2z) * [(C(w2)-C(w1)) + i(S(w2)-S(w1))],
      w1 = p*sqrt(2/z),  w2 = (p + z)*sqrt(2/z),

with C, S the Fresnel integrals (argument convention of scipy.special.fresnel:
C(x) = integral_0^x cos(pi t^2 / 2) dt).  For z < 0, A(q, z) = conj(A(-q, -z))
(substitute into the integral), and for z = 0 the integral is elementary:
A(q, 0) = exp(i*pi*q) * sinc(q).
"""

import numpy as np
from scipy.special import fresnel


def tap_count(z):
    """Taps of template z: L(z) = 2*(8 + ceil(4.5*|z|)), always even."""
    az = abs(int(z))
    return 2 * (8 + (9 * az + 1) // 2)


def tap_offsets(z):
    """Offsets d of template z, d in [-L/2, L/2 - 1] (centred support)."""
    half = tap_count(z) // 2
    return np.arange(-half, half, dtype=np.int64)


def _phase_p2_over_z(q, z):
    """exp(-i*pi*p^2/z) with p = q - z/2, for integer q and integer z > 0.

    p^2/z = (2q - z)^2 / (4z).  With n = (2q - z)^2 an exact integer the
    angle pi*n/(4z) is reduced modulo 2*pi (n mod 8z) before the float
    multiply, so the phase carries no error that grows with q.
    """
    n = (2 * q - z) ** 2
    red = np.mod(n, 8 * z).astype(np.float64)
    return np.exp(-1j * np.pi * red / (4.0 * z))


def response(q, z):
    """A(q, z) for integer arrays/scalars q and an integer z (closed form).

    q is the offset r_c - k in bins.  Only integer q is needed for templates
    (the oracle evaluates A at integer tap offsets).
    """
    q = np.asarray(q, dtype=np.int64)
    z = int(z)
    if z == 0:
        qf = q.astype(np.float64)
        # exp(i*pi*q) * sin(pi q)/(pi q); numpy's sinc is sin(pi x)/(pi x).
        return np.exp(1j * np.pi * np.mod(qf, 2.0)) * np.sinc(qf)
    if z < 0:
        return np.conj(response(-q, -z))
    p = q.astype(np.float64) - 0.5 * z
    s = np.sqrt(2.0 / z)
    S1, C1 = fresnel(p * s)
    S2, C2 = fresnel((p + z) * s)
    return _phase_p2_over_z(q, z) / np.sqrt(2.0 * z) * ((C2 - C1) + 1j * (S2 - S1))


def template(z):
    """(offsets d, complex128 taps h_z[d]) of unit energy."""
    d = tap_offsets(z)
    a = response(-d, z)
    energy = np.sum(np.abs(a) ** 2)
    return d, np.conj(a) / np.sqrt(energy)


def support_energy(z):
    """E_z = sum over the support of |A(-d, z)|^2 (fraction of the total, <= 1)."""
    d = tap_offsets(z)
    return float(np.sum(np.abs(response(-d, z)) ** 2))


def template_bank(z_max=42):
    """List of (z, offsets, taps) for z = -z_max .. z_max, in row order."""
    return [(z,) + template(z) for z in range(-z_max, z_max + 1)]
