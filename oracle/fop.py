"""FT convolution into the filter-output plane (oracle, FP64).

Test infrastructure only: imported by tests, the smoke check and the CPU
baseline of the benchmark, never by the library.

Section 2.1 applies N_temp FIR filters to the N_chan-point complex spectrum.
eq. (1) writes each filter as a direct complex FIR sum and eq. (2) as the
convolution theorem; the overlap-save form of Section 2.1.2 only splits the
same convolution into chunks.  Both reach the same plain definition, which is
what this module computes:

    y_z[j] = sum_{d=-L/2}^{L/2-1} X[j + d] * h_z[d],   X[k] = 0 outside [0, N)
    FOP[z + z_max][j] = |y_z[j]|^2                     (Section 2.2: the power
                                                        of the filter outputs)

Reading (the paper leaves the alignment of output column and bin open): the
filter is centred, so column j of the FOP is Fourier bin j.  This equals
eq. (1) with reversed taps and the output shifted by L/2.  Both ends of the
spectrum are zero-extended (Section 2.1.2 states the zero padding only for the
start), so every row has exactly N outputs.
"""

import numpy as np
import scipy.fft

from .response import template_bank


def correlate_direct(x, d, h):
    """y[j] = sum_d x[j + d] h[d], zero outside [0, N): the definition, O(N*L).

    Vectorised over j, one tap at a time; used as the brute-force pin and for
    sampled outputs at large N.
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    y = np.zeros(n, dtype=np.complex128)
    for dd, hh in zip(d.tolist(), h.tolist()):
        lo = max(0, -dd)
        hi = min(n, n - dd)
        if hi > lo:
            y[lo:hi] += x[lo + dd:hi + dd] * hh
    return y


def correlate_points(x, d, h, cols):
    """y[j] at selected columns only (direct sum per column)."""
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    cols = np.asarray(cols, dtype=np.int64)
    idx = cols[:, None] + d[None, :]
    ok = (idx >= 0) & (idx < n)
    xs = np.where(ok, x[np.clip(idx, 0, n - 1)], 0.0)
    return xs @ h


def _fft_len(n, half):
    return scipy.fft.next_fast_len(n + half + 1)


def correlate_fft(x, d, h, workers=None):
    """Same correlation through eq. (2): circular correlation of zero-padded data.

    With M >= N + L/2 + 1 and the taps placed at d mod M, the circular
    correlation sum_e xp[(j+e) mod M] hp[e mod M] never wraps for j in [0, N),
    so it equals the linear definition.  In the DFT domain a correlation with
    hp is a product with conj(DFT(conj(hp))).
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    half = int(max(-d.min(), d.max() + 1))
    m = _fft_len(n, half)
    xp = np.zeros(m, dtype=np.complex128)
    xp[:n] = x
    hp = np.zeros(m, dtype=np.complex128)
    hp[np.mod(d, m)] = h
    fx = scipy.fft.fft(xp, workers=workers)
    fh = np.conj(scipy.fft.fft(np.conj(hp), workers=workers))
    return scipy.fft.ifft(fx * fh, workers=workers)[:n]


def fop(x, z_max=42, method="fft", workers=None, dtype=np.float64):
    """Filter-output plane, shape (2*z_max+1, N): row z + z_max, column = bin.

    method "fft" uses eq. (2) (zero-padded FFT correlation), "direct" the sum
    of eq. (1).  One forward transform of the spectrum is shared by all
    templates, as in the AOLS design of Section 2.1.3.
    """
    x = np.asarray(x, dtype=np.complex128)
    n = x.shape[0]
    bank = template_bank(z_max)
    out = np.empty((len(bank), n), dtype=dtype)
    if method == "direct":
        for row, (_, d, h) in enumerate(bank):
            out[row] = np.abs(correlate_direct(x, d, h)) ** 2
        return out
    half = max(int(max(-d.min(), d.max() + 1)) for _, d, _ in bank)
    m = _fft_len(n, half)
    xp = np.zeros(m, dtype=np.complex128)
    xp[:n] = x
    fx = scipy.fft.fft(xp, workers=workers)
    for row, (_, d, h) in enumerate(bank):
        hp = np.zeros(m, dtype=np.complex128)
        hp[np.mod(d, m)] = h
        fh = np.conj(scipy.fft.fft(np.conj(hp), workers=workers))
        y = scipy.fft.ifft(fx * fh, workers=workers)[:n]
        out[row] = y.real ** 2 + y.imag ** 2
    return out


def fop_points(x, rows, cols, z_max=42):
    """FOP values at (row, col) pairs, each from the direct sum of eq. (1)."""
    bank = template_bank(z_max)
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    for r in np.unique(rows):
        sel = rows == r
        _, d, h = bank[int(r)]
        y = correlate_points(x, d, h, cols[sel])
        out[sel] = y.real ** 2 + y.imag ** 2
    return out
