"""GPU parity of the alternative harmonic index maps (plan option hsum_index).

FDAS_HSUM_FUNDAMENTAL: HP_k(i, j) = HP_{k-1}(i, j) + FOP(k i, k j), 0 outside.
FDAS_HSUM_HIGHEST:     HP_k(i, j) = sum_{m<=k} FOP(rho(m i, k), rho(m j, k)).

The kernels are fed the oracle's FOP rounded to FP32 and compared with the
oracle's FP32 twin (same summation order): candidate indices and power bits
identical.  End to end (GPU convolution + GPU harmonic sum) an injected
pulsar with integer (r, z) is recovered at the cells each map predicts.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import fop as ofop  # noqa: E402
from oracle import harmonic as oh  # noqa: E402
from paper_1806_01556_amd import fdas, synth  # noqa: E402

MAPS = {"fundamental": fdas.HSUM_FUNDAMENTAL, "highest": fdas.HSUM_HIGHEST}
_plans = {}


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def plan_for(index, z_max=42, n_harm=8, n_max=1 << 20):
    key = (index, z_max, n_harm, n_max)
    if key not in _plans:
        _plans[key] = fdas.plan_create(z_max=z_max, n_harm=n_harm, n_max=n_max, hsum_index=MAPS[index])
    return _plans[key]


def _upload_plane(plane32):
    rows, n = plane32.shape
    buf = np.zeros((rows, fdas.fop_ld(n)), dtype=np.float32)
    buf[:, :n] = plane32
    return torch.from_numpy(buf).to(_dev())


def gpu_candidates(plan, plane32, ta=None):
    n = plane32.shape[1]
    print(f"hsum index={plan.desc.hsum_index} n={n} z_max={plan.desc.z_max} n_harm={plan.desc.n_harm}", flush=True)
    cands, counts = fdas.alloc_cands(plan, _dev())
    ta_t = None if ta is None else torch.from_numpy(np.ascontiguousarray(ta, dtype=np.float32)).to(_dev())
    fdas.harmonic_sum(plan, _upload_plane(plane32), n, cands, counts, ta=ta_t)
    return fdas.candidates(plan, cands, counts)


def _assert_same(got, ref):
    assert got.size == ref.size, (got.size, ref.size)
    for f in ("harm", "z", "r"):
        assert np.array_equal(got[f], ref[f]), f
    assert np.array_equal(got["power"].astype(np.float32).view(np.int32),
                          ref["power"].astype(np.float32).view(np.int32))


@pytest.mark.parametrize("index", sorted(MAPS))
@pytest.mark.parametrize("n_harm", [1, 2, 3, 5, 8])
def test_bit_exact_on_oracle_fop(index, n_harm):
    plan = plan_for(index, n_harm=n_harm)
    spec, _ = synth.make_spectrum(1 << 16, 21, pulsars=[synth.Pulsar(r=12000.0, z=10.0, snr=12.0, n_harm=4)])
    plane = ofop.fop(spec.astype(np.complex128)).astype(np.float32)
    ta = oh.threshold_array(n_harm, 42, 2e-4).astype(np.float32)
    got, counts = gpu_candidates(plan, plane, ta=ta)
    ref = oh.candidates(plane, n_harm, ta=ta, index=index)
    assert np.array_equal(counts, oh.plane_counts(ref, n_harm))
    _assert_same(got, ref)


@pytest.mark.parametrize("index", sorted(MAPS))
@pytest.mark.parametrize("n", [1, 2, 3, 5, 57, 1001, 4099])
def test_ragged_and_tiny(index, n):
    plan = plan_for(index)
    rng = np.random.default_rng(n)
    plane = rng.exponential(size=(85, n)).astype(np.float32)
    ta = oh.threshold_array(8, 42, 0.02).astype(np.float32)
    got, _ = gpu_candidates(plan, plane, ta=ta)
    _assert_same(got, oh.candidates(plane, 8, ta=ta, index=index))


@pytest.mark.parametrize("index", sorted(MAPS))
@pytest.mark.parametrize("z_max", [0, 3, 10, 64])
def test_other_row_counts_and_row_dependent_ta(index, z_max):
    rows, n = 2 * z_max + 1, 3000
    plan = plan_for(index, z_max=z_max)
    rng = np.random.default_rng(100 + z_max)
    plane = rng.exponential(size=(rows, n)).astype(np.float32)
    ta = oh.threshold_array(8, z_max, 0.01).astype(np.float32)
    ta = ta * (1.0 + 0.01 * np.arange(rows, dtype=np.float32)[None, :])
    got, _ = gpu_candidates(plan, plane, ta=ta)
    _assert_same(got, oh.candidates(plane, 8, ta=ta, index=index))


@pytest.mark.parametrize("index", sorted(MAPS))
def test_large_plane_windows(index):
    # 2^20 columns in one launch; candidates compared in three column windows
    n = 1 << 20
    plan = plan_for(index)
    rng = np.random.default_rng(7)
    plane = rng.exponential(size=(85, n)).astype(np.float32)
    ta = oh.threshold_array(8, 42, 1e-4).astype(np.float32)  # ~9k cells per plane, under the list capacity
    got, _ = gpu_candidates(plan, plane, ta=ta)
    for lo, hi in [(0, 3000), (n // 2 - 1500, n // 2 + 1500), (n - 3000, n)]:
        cols = np.arange(lo, hi)
        ref = oh.candidates(plane, 8, ta=ta, cols=cols, index=index)
        sel = got[(got["r"] >= lo) & (got["r"] < hi)]
        _assert_same(sel, ref)


@pytest.mark.parametrize("index", sorted(MAPS))
def test_end_to_end_injection(index):
    r0, z0 = 12000, 10
    spec, _ = synth.make_spectrum(1 << 16, 21, pulsars=[synth.Pulsar(r=float(r0), z=float(z0), snr=12.0, n_harm=4)])
    n = spec.shape[0]
    plan = plan_for(index, n_max=1 << 16)
    x = torch.from_numpy(spec).to(_dev())
    got, _, fop_t = fdas.search(plan, x)
    plane = ofop.fop(spec.astype(np.complex128))
    ref = oh.candidates(plane, 8, index=index)
    guard = oh.guard_cells(plane, 8, index=index)
    gk = set(zip(got["harm"].tolist(), got["z"].tolist(), got["r"].tolist()))
    rk = set(zip(ref["harm"].tolist(), ref["z"].tolist(), ref["r"].tolist()))
    assert not (gk - rk - guard) and not (rk - gk - guard)
    for k in range(1, 5):
        cell = (k, z0, r0) if index == "fundamental" else (k, k * z0, k * r0)
        assert cell in gk, cell


@pytest.mark.parametrize("index", sorted(MAPS))
def test_dense_hits_and_capacity_overflow(index):
    # most cells above threshold: every wave appends many records per plane
    # at once; with a 16-record list the counts stay exact and the records
    # kept are true candidates
    n = 5000
    rng = np.random.default_rng(3)
    plane = (rng.exponential(size=(85, n)) * 5).astype(np.float32)
    ta = oh.threshold_array(8, 42, 0.01).astype(np.float32)
    ref = oh.candidates(plane, 8, ta=ta, index=index)
    big = fdas.plan_create(n_max=1 << 16, hsum_index=MAPS[index], cand_capacity=1 << 20)
    small = fdas.plan_create(n_max=1 << 16, hsum_index=MAPS[index], cand_capacity=16)
    try:
        got, counts = gpu_candidates(big, plane, ta=ta)
        assert np.array_equal(counts, oh.plane_counts(ref))
        _assert_same(got, ref)
        cands, dcounts = fdas.alloc_cands(small, _dev())
        fdas.harmonic_sum(small, _upload_plane(plane), n, cands, dcounts,
                          ta=torch.from_numpy(ta).to(_dev()))
        assert np.array_equal(dcounts.cpu().numpy(), oh.plane_counts(ref))
        kept, _ = fdas.candidates(small, cands, dcounts, allow_overflow=True)
        assert kept.size == 8 * 16
        refset = set(zip(ref["harm"].tolist(), ref["z"].tolist(), ref["r"].tolist(),
                         ref["power"].astype(np.float32).view(np.int32).tolist()))
        assert all(k in refset for k in zip(kept["harm"].tolist(), kept["z"].tolist(), kept["r"].tolist(),
                                            kept["power"].astype(np.float32).view(np.int32).tolist()))
    finally:
        big.destroy()
        small.destroy()


@pytest.mark.timeout(400)
@pytest.mark.parametrize("index", sorted(MAPS))
def test_wide_single_row_plane(index):
    # one template row (z_max = 0) admits spectra past 2^28 bins: the
    # highest-anchored map then rounds m j / k in its wide form and the
    # fundamental-anchored map's stride-k reads run past 2^31 bytes; three
    # column windows (start, the 2^28 boundary, end) against the oracle
    n = (1 << 28) + 5000
    plan = fdas.plan_create(z_max=0, n_max=n, hsum_index=MAPS[index], cand_capacity=1 << 20)
    try:
        rng = np.random.default_rng(28)
        plane = rng.standard_exponential(size=(1, n), dtype=np.float32)
        ta = oh.threshold_array(8, 0, 2e-3).astype(np.float32)  # ~0.5 M cells per plane
        got, _ = gpu_candidates(plan, plane, ta=ta)
        print(f"wide plane {index}: {got.size} candidates", flush=True)
        for lo, hi in [(0, 4000), ((1 << 28) - 3000, (1 << 28) + 1000), (n - 4000, n)]:
            cols = np.arange(lo, hi)
            ref = oh.candidates(plane, 8, ta=ta, cols=cols, index=index)
            sel = got[(got["r"] >= lo) & (got["r"] < hi)]
            assert ref.size > 5
            _assert_same(sel, ref)
    finally:
        plan.destroy()
