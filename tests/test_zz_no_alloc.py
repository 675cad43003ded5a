"""fdas_harmonic_sum_noalloc (scratch in the library's static device array,
no allocation) against fdas_harmonic_sum on the same FOP: identical counts,
candidate indices and power bits, on two calls in a row, the second with a
smaller input (the static array keeps the first call's contents), for the
85-row stretched sum, for a plan with another row count (the generic kernel,
which uses no scratch) and a row-dependent threshold array, for the two other
index maps (their tile order lives in the static array); n above the static
capacity is rejected before anything runs.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from paper_1806_01556_amd import fdas, synth  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def _readback(plan, cands, counts):
    c, hc = fdas.candidates(plan, cands, counts, allow_overflow=True)
    return c, hc


def _same(a, b):
    assert a.size == b.size, (a.size, b.size)
    for f in ("harm", "z", "r"):
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["power"].view(np.int32), b["power"].view(np.int32))


def _compare(plan, spec, ta=None):
    n = spec.shape[0]
    x = torch.from_numpy(spec).to(_dev())
    fop = fdas.alloc_fop(plan, n, _dev())
    print(f"no-alloc: convolve n={n} z_max={plan.desc.z_max}", flush=True)
    fdas.convolve(plan, x, fop, n=n)
    ta_t = None if ta is None else torch.from_numpy(np.ascontiguousarray(ta, dtype=np.float32)).to(_dev())
    c1, k1 = fdas.alloc_cands(plan, _dev())
    fdas.harmonic_sum(plan, fop, n, c1, k1, ta=ta_t)
    ref, hr = _readback(plan, c1, k1)
    c2, k2 = fdas.alloc_cands(plan, _dev())
    k2.fill_(-7)  # the call must reset the counts itself
    print(f"no-alloc: harmonic_sum_noalloc n={n}", flush=True)
    fdas.harmonic_sum_noalloc(plan, fop, n, c2, k2, ta=ta_t)
    got, hg = _readback(plan, c2, k2)
    assert np.array_equal(hr, hg), (hr, hg)
    _same(got, ref)
    return got.size


def test_noalloc_equals_harmonic_sum_two_calls_second_smaller():
    plan = fdas.plan_create(n_max=1 << 22)
    try:
        big, _ = synth.ska(n=1 << 22, seed=2)
        nb = _compare(plan, big)
        small, _ = synth.make_spectrum(300_001, 71, n_random=3, r_range=(2000, 1.2e5), snr_range=(8, 20))
        ns = _compare(plan, small)
        print(f"no-alloc: {nb} and {ns} candidates identical", flush=True)
        assert nb > ns > 0
    finally:
        plan.destroy()


def test_noalloc_generic_rows_and_row_dependent_thresholds():
    plan = fdas.plan_create(n_max=1 << 17, z_max=5)
    try:
        spec, _ = synth.make_spectrum(100_003, 72, n_random=3, r_range=(500, 4e4), snr_range=(8, 20))
        ta = fdas.thresholds(8, 1e-4).astype(np.float32)[:, None] * (1.0 + 0.01 * np.arange(11, dtype=np.float32))
        _compare(plan, spec, ta=ta)
        spec2, _ = synth.make_spectrum(5001, 73, n_random=1, r_range=(500, 2000), snr_range=(8, 20))
        _compare(plan, spec2)
    finally:
        plan.destroy()


@pytest.mark.parametrize("index", [fdas.HSUM_FUNDAMENTAL, fdas.HSUM_HIGHEST])
def test_noalloc_other_index_maps(index):
    # the index-map kernels take their tile order from the static array too
    plan = fdas.plan_create(n_max=1 << 22, hsum_index=index)
    try:
        big, _ = synth.ska(n=1 << 22, seed=2)
        nb = _compare(plan, big)
        small, _ = synth.make_spectrum(300_001, 74, n_random=3, r_range=(2000, 1.2e5), snr_range=(8, 20))
        ns = _compare(plan, small)
        assert nb > 0 and ns > 0
    finally:
        plan.destroy()


def test_noalloc_rejects_n_beyond_its_scratch():
    plan = fdas.plan_create(n_max=(1 << 22) + 64)
    try:
        n = (1 << 22) + 4
        fop = torch.zeros((85, n), dtype=torch.float32, device=_dev())
        cands, counts = fdas.alloc_cands(plan, _dev())
        with pytest.raises(fdas.FdasError) as e:
            fdas.harmonic_sum_noalloc(plan, fop, n, cands, counts)
        assert e.value.status == fdas.ERR_INVALID_ARG
        assert "static scratch" in str(e.value)
    finally:
        plan.destroy()
