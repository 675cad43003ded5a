"""CPU FP64 oracle for the FDAS hot path (test infrastructure only).

This package is the reference against which the GPU library is checked.  It
is plain NumPy/SciPy in float64, written for readability, not speed, and it
shares no code, table or constant generator with the HIP library.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import it.  The product path never calls it.

What it computes (Wang, Thiagaraj & Sinnen, "Combining Multiple Optimized
FPGA-based Pulsar Search Modules Using OpenCL"):

* ``response``  -- the Fourier-domain response of a constant-fdot signal and
  the 85 acceleration templates built from it (the template formula is not
  printed in the paper; it follows the Ransom et al. acceleration search that
  the paper's introduction names as the basis of FDAS).
* ``fop``       -- the FT-convolution step of Section 2.1: every template
  correlated with the spectrum (eq. (1), equivalently eq. (2)) and the power
  of each output, giving the filter-output plane (FOP).
* ``harmonic``  -- the harmonic-summing step of Section 2.2 (Algorithm 1):
  stretch planes, cumulative harmonic planes, per-plane thresholds and the
  candidate list.
* ``prescreen`` -- not from the paper: the small 1D convolutional network of
  the learned block pre-screen (forward, loss and backward in float64), the
  reference for the GPU training and inference kernels.

Every function states the passage it follows.  Readings of passages the
paper leaves open are stated where they are used and collected in the
design notes of the repository.
"""

from . import response, fop, harmonic, prescreen  # noqa: F401
