"""Seeded synthetic spectra for the FDAS hot path.

This module only makes inputs: complex Gaussian noise plus drifting
sinusoids (pulsars) injected in the time domain and Fourier transformed in
FP64.  It holds none of the search's arithmetic (no templates, correlation or
harmonic sums), so the GPU library and the CPU oracle can both be fed from it.

Conventions
-----------
* Noise: Re, Im ~ N(0, 1/2) independently, so E|X|^2 = 1 per bin.
* A pulsar has mean Fourier frequency r (bins), total drift z (bins over the
  observation), amplitude SNR ``snr`` and ``n_harm`` harmonics.  Harmonic h
  has mean frequency h*r, drift h*z, amplitude snr/h and a random phase.  It
  is synthesised as the time series
      x_n = (snr/h)/N * exp(2*pi*i*(h*(r*u + z*(u^2 - u)/2)) + i*psi),  u = n/N,
  and added to the spectrum through an FP64 DFT X[k] = sum_n x_n e^{-2 pi i nk/N}.
  With that normalisation the noise-free matched-filter power of a
  unit-energy template centred on (r, z) is about snr^2 (amplitude SNR).
* A harmonic whose band [h*r - |h*z|/2, h*r + |h*z|/2] comes within 64 bins of
  either end of the spectrum is skipped (it would alias).
* Draw order from numpy PCG64(seed): noise (2N normals), then the pulsar
  parameters (when drawn at random), then one phase per harmonic.

Workloads (sizes follow Table 1 of the paper: 85 templates, 8 harmonic
planes; the spectrum length is 2^16 for the small case and 2^22 for the
SKA-sized case):
* ``plain``    N = 2^16, seed 1, one pulsar r = 20000.3, z = 17.5, SNR 10,
               4 harmonics.
* ``ska``      N = 2^22, seed 2, 16 pulsars with r ~ U[1e4, 2e6],
               z ~ U[-42, 42], SNR ~ U[6, 20], harmonics ~ U{1..8}.
* ``batch``    spectrum b of a batch: seed 3000 + b, N drawn from
               {2^20, 2^21, 3*2^20, 2^22}, 0-4 pulsars with r ~ U[1e4, 0.45 N].
"""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Pulsar:
    r: float
    z: float
    snr: float
    n_harm: int
    phases: list = field(default_factory=list)
    injected: list = field(default_factory=list)  # harmonics actually added


def _rng(seed):
    return np.random.Generator(np.random.PCG64(int(seed)))


def noise(n, rng):
    """Unit-variance complex Gaussian noise, Re/Im ~ N(0, 1/2), complex128."""
    v = rng.standard_normal(2 * n).reshape(n, 2) * np.sqrt(0.5)
    return v[:, 0] + 1j * v[:, 1]


def _chirp_series(n, r, z, amp, psi):
    """x_n = amp/N * exp(2 pi i (r u + z (u^2 - u)/2) + i psi), u = n/N (FP64)."""
    k = np.arange(n, dtype=np.float64)
    u = k / n
    cycles = r * u + 0.5 * z * (u * u - u)
    cycles = cycles - np.floor(cycles)
    return (amp / n) * np.exp(1j * (2.0 * np.pi * cycles + psi))


def inject(spec, pulsars, rng):
    """Add the pulsars' harmonics to ``spec`` (complex128, modified in place)."""
    n = spec.shape[0]
    series = np.zeros(n, dtype=np.complex128)
    any_added = False
    for p in pulsars:
        p.phases = list(rng.uniform(0.0, 2.0 * np.pi, size=p.n_harm))
        p.injected = []
        for h in range(1, p.n_harm + 1):
            hr, hz = h * p.r, h * p.z
            lo, hi = hr - 0.5 * abs(hz), hr + 0.5 * abs(hz)
            if lo < 64 or hi > n - 64:
                continue
            series += _chirp_series(n, hr, hz, p.snr / h, p.phases[h - 1])
            p.injected.append(h)
            any_added = True
    if any_added:
        spec += np.fft.fft(series)
    return spec


def make_spectrum(n, seed, pulsars=None, n_random=0, r_range=(1e4, 2e6),
                  z_range=(-42.0, 42.0), snr_range=(6.0, 20.0), harm_range=(1, 8)):
    """Seeded spectrum: (complex64[n], list of Pulsar).

    ``pulsars`` gives fixed pulsars; otherwise ``n_random`` are drawn.
    """
    rng = _rng(seed)
    spec = noise(n, rng)
    if pulsars is None:
        pulsars = []
        for _ in range(n_random):
            r = rng.uniform(*r_range)
            z = rng.uniform(*z_range)
            snr = rng.uniform(*snr_range)
            nh = int(rng.integers(harm_range[0], harm_range[1] + 1))
            pulsars.append(Pulsar(r=r, z=z, snr=snr, n_harm=nh))
    inject(spec, pulsars, rng)
    return spec.astype(np.complex64), pulsars


def plain(n=1 << 16, seed=1):
    """Small single spectrum: one pulsar r=20000.3, z=17.5, SNR 10, 4 harmonics."""
    return make_spectrum(n, seed, pulsars=[Pulsar(r=20000.3, z=17.5, snr=10.0, n_harm=4)])


def ska(n=1 << 22, seed=2, n_pulsars=16):
    """SKA-sized spectrum: 16 random pulsars (see module docstring)."""
    return make_spectrum(n, seed, n_random=n_pulsars, r_range=(1e4, 2e6))


BATCH_LENGTHS = (1 << 20, 1 << 21, 3 << 20, 1 << 22)


def batch_member(b, base_seed=3000):
    """Spectrum b of a batch of uneven lengths (see module docstring)."""
    rng = _rng(base_seed + b)
    n = int(BATCH_LENGTHS[int(rng.integers(0, len(BATCH_LENGTHS)))])
    n_p = int(rng.integers(0, 5))
    seed = int(rng.integers(0, 2**31 - 1))
    return make_spectrum(n, seed, n_random=n_p, r_range=(1e4, 0.45 * n))


def noise_only(n, seed):
    """Pure noise spectrum (complex64)."""
    return noise(n, _rng(seed)).astype(np.complex64)
