"""GPU parity of the direct (matrix-core) correlation against the CPU oracle.

fdas_convolve with method FDAS_CONV_DIRECT_MFMA computes the same plane as the
overlap-save method (eq. (1) of Section 2.1 evaluated as a sum over taps), so
it is held to the same bound: |P - P_ref| <= 1e-4 * max(P_ref, 1) for every
cell, against the FP64 oracle.  The kernel works on 512-bin workgroups and
tiles of 8 templates grouped by |z|, so the lengths below cover one partial
workgroup, exact multiples, ragged tails and several workgroups; the template
counts cover a partial last tile (z_max = 42: 85 = 10 * 8 + 5), a single
template, and the widest templates the plan accepts (z_max = 64).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import skaref  # noqa: E402
from oracle import fop as ofop  # noqa: E402
from oracle import harmonic as oh  # noqa: E402
from paper_1806_01556_amd import fdas, synth  # noqa: E402

TOL = 1e-4
_plans = {}


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def direct_plan(z_max=42, n_max=1 << 22):
    key = (z_max, n_max)
    if key not in _plans:
        _plans[key] = fdas.plan_create(z_max=z_max, n_max=n_max, method=fdas.CONV_DIRECT_MFMA)
    return _plans[key]


def gpu_fop(plan, spec):
    n = spec.shape[0]
    x = torch.from_numpy(np.ascontiguousarray(spec.astype(np.complex64))).to(_dev())
    out = torch.full((plan.rows, fdas.fop_ld(n)), float("nan"), dtype=torch.float32, device=_dev())
    print(f"direct convolve: n={n} z_max={plan.desc.z_max}", flush=True)
    fdas.convolve(plan, x, out, n=n)
    torch.cuda.synchronize()
    return out


def assert_fop_close(got, ref):
    err = np.abs(got.astype(np.float64) - ref)
    bound = TOL * np.maximum(ref, 1.0)
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} cells off; worst ratio {np.max(err / bound):.3g}"
    return float(np.max(err / bound))


@pytest.mark.parametrize("n", [1, 3, 100, 511, 512, 513, 1024, 4099, 12345])
def test_direct_ragged_lengths(n):
    plan = direct_plan()
    spec, _ = synth.make_spectrum(n, 300 + n)
    got = gpu_fop(plan, spec).cpu().numpy()
    ref = ofop.fop(spec.astype(np.complex128))
    assert_fop_close(got[:, :n], ref)
    assert np.all(np.isnan(got[:, n:])), "columns >= n must not be written"


@pytest.mark.parametrize("z_max", [0, 1, 5, 17, 64])
def test_direct_other_template_counts(z_max):
    n = 9000
    plan = direct_plan(z_max=z_max, n_max=1 << 16)
    spec, _ = synth.make_spectrum(n, 17 + z_max, n_random=2, r_range=(500, 8000))
    got = gpu_fop(plan, spec).cpu().numpy()[:, :n]
    assert_fop_close(got, ofop.fop(spec.astype(np.complex128), z_max=z_max))


def test_direct_plain_workload_full_plane_and_candidates():
    plan = direct_plan()
    spec, _ = synth.plain()
    n = spec.shape[0]
    fop_t = gpu_fop(plan, spec)
    got = fop_t.cpu().numpy()[:, :n]
    ref = ofop.fop(spec.astype(np.complex128))
    worst = assert_fop_close(got, ref)
    print(f"direct, plain 2^16: worst |err|/bound = {worst:.3g}", flush=True)
    # candidates from the direct plane: identical outside the guard band
    cands, counts = fdas.alloc_cands(plan, _dev())
    fdas.harmonic_sum(plan, fop_t, n, cands, counts)
    c, _ = fdas.candidates(plan, cands, counts)
    rc = oh.candidates(ref, 8)
    guard = oh.guard_cells(ref, 8)
    gk = set(zip(c["harm"].tolist(), c["z"].tolist(), c["r"].tolist()))
    rk = set(zip(rc["harm"].tolist(), rc["z"].tolist(), rc["r"].tolist()))
    assert not (gk - rk - guard) and not (rk - gk - guard)
    assert (1, 17, 20000) in gk or (1, 18, 20000) in gk


@pytest.mark.timeout(900)
def test_direct_ska_size_full_plane():
    # full SKA length in one launch: every one of the 85 x 2^22 cells against
    # the FP64 oracle, plus workgroup-boundary columns against the direct sum
    plan = direct_plan()
    spec, _, plane64, _, _, _ = skaref.ska()
    n = spec.shape[0]
    got = gpu_fop(plan, spec).cpu().numpy()
    worst = skaref.assert_plane_close(got, plane64)
    print(f"direct, ska 2^22, all {85 * n} cells: worst |err|/bound = {worst:.3g}", flush=True)
    cc = np.repeat(np.array([0, 511, 512, 4095 * 512 - 1, 4095 * 512, n - 1]), 85)
    rr = np.tile(np.arange(85), 6)
    assert_fop_close(got[rr, cc], ofop.fop_points(spec.astype(np.complex128), rr, cc))


def test_direct_matches_overlap_save():
    # both methods compute the same correlation; each is within 1e-4 of the
    # oracle, so they agree within twice that
    n = 40000
    spec, _ = synth.make_spectrum(n, 4242, n_random=4, r_range=(1000, 30000))
    a = gpu_fop(direct_plan(), spec).cpu().numpy()[:, :n].astype(np.float64)
    ols = fdas.plan_create(n_max=1 << 16, method=fdas.CONV_OLS_FFT)
    try:
        x = torch.from_numpy(spec.astype(np.complex64)).to(_dev())
        out = torch.empty((85, fdas.fop_ld(n)), dtype=torch.float32, device=_dev())
        fdas.convolve(ols, x, out, n=n)
        torch.cuda.synchronize()
        b = out.cpu().numpy()[:, :n].astype(np.float64)
    finally:
        ols.destroy()
    assert np.max(np.abs(a - b) / np.maximum(np.maximum(a, b), 1.0)) < 2 * TOL
