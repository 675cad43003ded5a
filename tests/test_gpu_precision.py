"""Split-precision direct correlation (FDAS_PREC_SPLIT_FP16 / _BF16) against the FP64 oracle.

Every operand value v is carried as hi = round16(v), lo = round16(v - hi) and
each product as hi*hi + hi*lo + lo*hi with FP32 accumulation.

Error bounds (from the arithmetic, for y = sum_d X[j+d] h[d] over L <= 394
taps, S = sum_d |X[j+d]| |h[d]|):
* FP16 split: hi + lo carries 22 significant bits and the dropped lo*lo term is
  ~2^-22 of a product, so |dy| is a few 2^-22 S, as for FP32; the FP32 power
  bound |dP| <= 1e-4 max(P, 1) applies unchanged.
* BF16 split: hi + lo carries 16 bits and lo*lo is ~2^-16 of a product:
  |dy| <~ 2^-15 S.  For noise-like input S ~ sqrt(L) |y|_rms, giving
  |dP| / max(P, 1) up to ~2 * 2^-15 * sqrt(394) ~ 1.2e-3; the test bound is
  4e-3 (the FP32 1e-4 bound is not met by BF16, which is why it cannot
  replace the FP32 path).
The per-template worst relative power error on sampled cells of SKA-sized
spectra is printed for FP16 split, BF16 split, FP32 direct and FP32
overlap-save; with FDAS_PRECISION_FULL=1 the same report covers every cell of
the 16 spectra of 2^22 bins of the precision workload (seeds 4000 + s; about
ten minutes of FP64 oracle time on 16 threads, so it is not part of the
default run).
"""

import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import skaref  # noqa: E402
from oracle import fop as ofop  # noqa: E402
from oracle import harmonic as oh  # noqa: E402
from paper_1806_01556_amd import fdas, synth  # noqa: E402

BOUND = {"fp16": 1e-4, "bf16": 4e-3}
PREC = {"fp16": fdas.PREC_SPLIT_FP16, "bf16": fdas.PREC_SPLIT_BF16}
_plans = {}


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


def plan_for(prec, z_max=42, n_max=1 << 22):
    key = (prec, z_max, n_max)
    if key not in _plans:
        if prec == "ols":
            _plans[key] = fdas.plan_create(z_max=z_max, n_max=n_max, method=fdas.CONV_OLS_FFT)
        elif prec == "fp32":
            _plans[key] = fdas.plan_create(z_max=z_max, n_max=n_max, method=fdas.CONV_DIRECT_MFMA)
        else:
            _plans[key] = fdas.plan_create(z_max=z_max, n_max=n_max, method=fdas.CONV_DIRECT_MFMA, precision=PREC[prec])
    return _plans[key]


def gpu_fop(plan, spec):
    n = spec.shape[0]
    x = torch.from_numpy(np.ascontiguousarray(spec.astype(np.complex64))).to(_dev())
    out = torch.full((plan.rows, fdas.fop_ld(n)), float("nan"), dtype=torch.float32, device=_dev())
    print(f"convolve: n={n} z_max={plan.desc.z_max} method={plan.desc.method} precision={plan.desc.precision}",
          flush=True)
    fdas.convolve(plan, x, out, n=n)
    torch.cuda.synchronize()
    return out


def rel_err(got, ref):
    return np.abs(got.astype(np.float64) - ref) / np.maximum(ref, 1.0)


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("n", [1, 3, 511, 512, 513, 4099, 12345])
def test_split_ragged_lengths(prec, n):
    plan = plan_for(prec)
    spec, _ = synth.make_spectrum(n, 700 + n)
    got = gpu_fop(plan, spec).cpu().numpy()
    err = rel_err(got[:, :n], ofop.fop(spec.astype(np.complex128)))
    assert err.max() <= BOUND[prec], f"{prec}: worst {err.max():.3g}"
    assert np.all(np.isnan(got[:, n:]))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("z_max", [0, 5, 64])
def test_split_other_template_counts(prec, z_max):
    n = 9000
    plan = plan_for(prec, z_max=z_max, n_max=1 << 16)
    spec, _ = synth.make_spectrum(n, 31 + z_max, n_random=2, r_range=(500, 8000))
    err = rel_err(gpu_fop(plan, spec).cpu().numpy()[:, :n], ofop.fop(spec.astype(np.complex128), z_max=z_max))
    assert err.max() <= BOUND[prec], f"{prec}: worst {err.max():.3g}"


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
def test_split_plain_workload_and_candidates(prec):
    plan = plan_for(prec)
    spec, _ = synth.plain()
    n = spec.shape[0]
    fop_t = gpu_fop(plan, spec)
    ref = ofop.fop(spec.astype(np.complex128))
    err = rel_err(fop_t.cpu().numpy()[:, :n], ref)
    print(f"{prec} split, plain 2^16: worst relative power error {err.max():.3g}", flush=True)
    assert err.max() <= BOUND[prec]
    cands, counts = fdas.alloc_cands(plan, _dev())
    fdas.harmonic_sum(plan, fop_t, n, cands, counts)
    c, _ = fdas.candidates(plan, cands, counts)
    rc = oh.candidates(ref, 8)
    guard = oh.guard_cells(ref, 8, rel=BOUND[prec])
    gk = set(zip(c["harm"].tolist(), c["z"].tolist(), c["r"].tolist()))
    rk = set(zip(rc["harm"].tolist(), rc["z"].tolist(), rc["r"].tolist()))
    assert not (gk - rk - guard) and not (rk - gk - guard)


def test_split_handles_tiny_magnitudes():
    # the whole spectrum scaled by 1e-6: unscaled FP16 operands would be
    # subnormal (a few significant bits); the power-of-two scaling of strips
    # and template tiles must keep the split errors at their normal level
    n = 20000
    spec, _ = synth.make_spectrum(n, 5, pulsars=[synth.Pulsar(r=6000.0, z=3.0, snr=30.0, n_harm=1)])
    spec = (spec * np.float32(1e-6)).astype(np.complex64)
    ref = ofop.fop(spec.astype(np.complex128))
    floor = 1e-12  # noise mean of the scaled spectrum
    worst = {}
    for prec in ("fp32", "fp16", "bf16"):
        got = gpu_fop(plan_for(prec), spec).cpu().numpy()[:, :n].astype(np.float64)
        worst[prec] = float(np.max(np.abs(got - ref) / np.maximum(ref, floor)))
    print("tiny magnitudes, worst relative power error:", worst, flush=True)
    assert worst["fp32"] <= 1e-4
    assert worst["fp16"] <= BOUND["fp16"]
    assert worst["bf16"] <= BOUND["bf16"]


def test_per_template_error_report_ska_size():
    # 4 SKA-sized spectra (the precision workload uses 16; sampled cells keep
    # the oracle's direct sums short), every method, worst error per template
    rng = np.random.default_rng(44)
    methods = ["fp16", "bf16", "fp32", "ols"]
    worst = {m: np.zeros(85) for m in methods}
    for sidx in range(4):
        spec, _ = synth.make_spectrum(1 << 22, 4000 + sidx, n_random=16, r_range=(1e4, 2e6))
        n = spec.shape[0]
        cols = np.concatenate([rng.integers(0, n, 96), [0, n - 1]])
        rows = np.repeat(np.arange(85), cols.size)
        cc = np.tile(cols, 85)
        ref = ofop.fop_points(spec.astype(np.complex128), rows, cc)
        for m in methods:
            got = gpu_fop(plan_for(m), spec).cpu().numpy()[rows, cc]
            e = rel_err(got, ref).reshape(85, cols.size).max(axis=1)
            worst[m] = np.maximum(worst[m], e)
    print("worst relative power error per template (z = -42..42), sampled cells of 4 x 2^22 spectra:")
    for m in methods:
        print(f"  {m:5s} max {worst[m].max():.3g}  median {np.median(worst[m]):.3g}  per z: "
              + " ".join(f"{v:.2g}" for v in worst[m]), flush=True)
    assert worst["fp16"].max() <= BOUND["fp16"]
    assert worst["bf16"].max() <= BOUND["bf16"]
    assert worst["fp32"].max() <= 1e-4 and worst["ols"].max() <= 1e-4


@pytest.mark.timeout(3000)
@pytest.mark.skipif(os.environ.get("FDAS_PRECISION_FULL") != "1",
                    reason="16 full 2^22-bin oracle planes (~10 min of CPU); set FDAS_PRECISION_FULL=1")
def test_per_template_error_report_full_precision_workload():
    """The precision workload at its stated size: 16 spectra of 2^22 bins
    (seeds 4000 + s, 16 pulsars each), every one of the 85 x 2^22 cells of
    each, worst |P - P_ref| / max(P_ref, 1) per template against the FP64
    oracle plane, for the split FP16 / BF16 and FP32 direct contractions and
    the FP32 overlap-save path."""
    methods = ["fp16", "bf16", "fp32", "ols"]
    worst = {m: np.zeros(85) for m in methods}
    cells = 0
    for sidx in range(16):
        spec, _ = synth.make_spectrum(1 << 22, 4000 + sidx, n_random=16, r_range=(1e4, 2e6))
        n = spec.shape[0]
        print(f"precision workload: spectrum {sidx + 1}/16, FP64 oracle plane", flush=True)
        ref = ofop.fop(spec.astype(np.complex128), workers=skaref.cpu_workers())
        for m in methods:
            got = gpu_fop(plan_for(m), spec).cpu().numpy()
            for r0 in range(0, 85, 5):
                g = got[r0:r0 + 5, :n].astype(np.float64)
                f = ref[r0:r0 + 5]
                worst[m][r0:r0 + 5] = np.maximum(worst[m][r0:r0 + 5],
                                                 np.max(np.abs(g - f) / np.maximum(f, 1.0), axis=1))
            del got
        cells += 85 * n
        del ref
        print(f"  worst so far: " + ", ".join(f"{m} {worst[m].max():.3g}" for m in methods), flush=True)
    print(f"worst relative power error per template (z = -42..42), every cell of 16 x 2^22 spectra "
          f"({cells} cells per method):")
    for m in methods:
        print(f"  {m:5s} max {worst[m].max():.3g}  median {np.median(worst[m]):.3g}  per z: "
              + " ".join(f"{v:.2g}" for v in worst[m]), flush=True)
    assert worst["fp16"].max() <= BOUND["fp16"]
    assert worst["bf16"].max() <= BOUND["bf16"]
    assert worst["fp32"].max() <= 1e-4 and worst["ols"].max() <= 1e-4
