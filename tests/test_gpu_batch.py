"""GPU tests of the batch path (fdas_search_batch / fdas_candidates_batch).

The batch path runs the same arithmetic as the single-spectrum calls (one
persistent convolution over a queue of (trial, chunk, template group) items,
one harmonic sum over every trial's tiles, replayed from a HIP graph), so its
FOPs and candidate lists must be bit-identical to fdas_convolve +
fdas_harmonic_sum + fdas_candidates on each trial, whatever the launch
parameters; and the candidates must match the FP64 oracle outside the guard
band.  Lengths are uneven and ragged (1 bin up to several chunks and tiles).
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import fop as ofop  # noqa: E402
from oracle import harmonic as oh  # noqa: E402
from paper_1806_01556_amd import fdas, synth  # noqa: E402

LENGTHS = [1, 1000, 3703, 3704, 4096, 12345, 40000, 65536, 100000]


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda:0")


class Batch:
    """Device buffers of a batch of trials and its Trial array."""

    def __init__(self, plan, specs):
        self.plan = plan
        self.specs = specs
        self.x = [torch.from_numpy(np.ascontiguousarray(s.astype(np.complex64))).to(_dev()) for s in specs]
        self.fop = [torch.full((plan.rows, fdas.fop_ld(s.shape[0])), float("nan"), dtype=torch.float32,
                               device=_dev()) for s in specs]
        self.cands = [fdas.alloc_cands(plan, _dev()) for _ in specs]
        self.trials = fdas.trials_array([(x, s.shape[0], f, f.shape[1], c[0], c[1])
                                         for x, s, f, c in zip(self.x, specs, self.fop, self.cands)])

    def run(self):
        print(f"search_batch: {len(self.specs)} trials, lengths {[s.shape[0] for s in self.specs]}", flush=True)
        fdas.search_batch(self.plan, self.trials)
        return fdas.candidates_batch(self.plan, self.trials)


def _specs(lengths, seed0):
    out = []
    for i, n in enumerate(lengths):
        if n >= 20000:
            s, _ = synth.make_spectrum(n, seed0 + i, n_random=2, r_range=(1000, n * 0.4), snr_range=(8.0, 20.0))
        else:
            s, _ = synth.make_spectrum(n, seed0 + i)
        out.append(s)
    return out


def _single(plan, spec):
    n = spec.shape[0]
    x = torch.from_numpy(spec.astype(np.complex64)).to(_dev())
    fop = torch.full((plan.rows, fdas.fop_ld(n)), float("nan"), dtype=torch.float32, device=_dev())
    cands, counts = fdas.alloc_cands(plan, _dev())
    fdas.convolve(plan, x, fop, n=n)
    fdas.harmonic_sum(plan, fop, n, cands, counts)
    c, hc = fdas.candidates(plan, cands, counts)
    return fop, c, hc


def _same(a, b):
    assert a.size == b.size, (a.size, b.size)
    for f in ("harm", "z", "r"):
        assert np.array_equal(a[f], b[f]), f
    assert np.array_equal(a["power"].view(np.int32), b["power"].view(np.int32))


_plan = None


def plan42():
    global _plan
    if _plan is None:
        _plan = fdas.plan_create(n_max=1 << 22)
    return _plan


@pytest.mark.parametrize("tuning", [{}, {"overlap_groups": 2}, {"overlap_groups": 3, "conv_templates_per_item": 9},
                                    {"conv_waves_per_simd": 1, "conv_templates_per_item": 85,
                                     "emit_workgroups": 256},
                                    {"hsum_tile": 256}, {"hsum_tile": 512, "overlap_groups": 2},
                                    {"ols_chunk": 4096, "hsum_tile": 1024}])
def test_batch_matches_single_calls_bit_for_bit(tuning):
    plan = plan42()
    fdas.set_tuning(plan, **tuning)
    try:
        specs = _specs(LENGTHS, 500)
        b = Batch(plan, specs)
        got, counts = b.run()
        for i, s in enumerate(specs):
            n = s.shape[0]
            fop1, c1, hc1 = _single(plan, s)
            assert torch.equal(b.fop[i][:, :n], fop1[:, :n]), f"trial {i} (n={n}): FOP differs"
            assert torch.all(torch.isnan(b.fop[i][:, n:])), "columns >= n must not be written"
            _same(got[i], c1)
            assert np.array_equal(counts[i], hc1)
    finally:
        fdas.set_tuning(plan)


def test_batch_candidates_match_oracle():
    plan = plan42()
    specs = _specs([3000, 50000, 65536], 900)
    got, _ = Batch(plan, specs).run()
    for i, s in enumerate(specs):
        plane = ofop.fop(s.astype(np.complex128))
        ref = oh.candidates(plane, 8)
        guard = oh.guard_cells(plane, 8)
        gk = set(zip(got[i]["harm"].tolist(), got[i]["z"].tolist(), got[i]["r"].tolist()))
        rk = set(zip(ref["harm"].tolist(), ref["z"].tolist(), ref["r"].tolist()))
        assert not (gk - rk - guard) and not (rk - gk - guard), i


def test_graph_replay_with_new_data_and_new_shapes():
    plan = plan42()
    shape_a = [5000, 70000, 12345]
    for rep, (lengths, seed) in enumerate([(shape_a, 10), (shape_a, 20), ([7000, 3], 30), (shape_a, 40)]):
        specs = _specs(lengths, seed)
        got, _ = Batch(plan, specs).run()
        for i, s in enumerate(specs):
            _, c1, _ = _single(plan, s)
            _same(got[i], c1)


def test_large_trials_sampled_against_oracle():
    # SKA-sized trials in one batch: sampled FOP cells against the direct sum
    plan = plan42()
    specs = [synth.batch_member(b)[0] for b in range(3)]
    b = Batch(plan, specs)
    got, counts = b.run()
    rng = np.random.default_rng(3)
    for i, s in enumerate(specs):
        n = s.shape[0]
        cols = np.concatenate([rng.integers(0, n, 300), [0, n - 1]])
        rows = rng.integers(0, 85, cols.size)
        ref = ofop.fop_points(s.astype(np.complex128), rows, cols)
        gotp = b.fop[i].cpu().numpy()[rows, cols].astype(np.float64)
        assert np.all(np.abs(gotp - ref) <= 1e-4 * np.maximum(ref, 1.0)), i
        _, c1, hc1 = _single(plan, s)
        _same(got[i], c1)
        assert np.array_equal(counts[i], hc1)


def test_top_k_per_trial():
    plan = fdas.plan_create(n_max=1 << 17, top_k=20)
    try:
        specs = _specs([40000, 100000], 77)
        got, counts = Batch(plan, specs).run()
        for i, s in enumerate(specs):
            _, c1, _ = _single(plan, s)
            _same(got[i], c1)
            assert all(np.sum(got[i]["harm"] == k) <= 20 for k in range(1, 9))
    finally:
        plan.destroy()


@pytest.mark.parametrize("kind", ["direct", "z_max_5", "fundamental"])
def test_batch_on_plans_without_the_graphed_path(kind):
    kw = {"direct": {"method": fdas.CONV_DIRECT_MFMA}, "z_max_5": {"z_max": 5},
          "fundamental": {"hsum_index": fdas.HSUM_FUNDAMENTAL}}[kind]
    plan = fdas.plan_create(n_max=1 << 17, **kw)
    try:
        specs = _specs([1000, 40000, 3703], 55)
        b = Batch(plan, specs)
        got, _ = b.run()
        for i, s in enumerate(specs):
            n = s.shape[0]
            fop1, c1, _ = _single(plan, s)
            assert torch.equal(b.fop[i][:, :n], fop1[:, :n])
            _same(got[i], c1)
    finally:
        plan.destroy()


@pytest.mark.parametrize("chunk", [2048, 8192])
def test_batch_at_other_chunk_lengths_matches_single_calls(chunk):
    """The batch at chunk length C equals the single calls of a plan built for
    C bit for bit, for every tile width."""
    plan = fdas.plan_create(n_max=1 << 17, ols_chunk=chunk)
    try:
        specs = _specs(LENGTHS, 700 + chunk)
        for tile in (256, 1024):
            fdas.set_tuning(plan, ols_chunk=chunk, hsum_tile=tile)
            b = Batch(plan, specs)
            got, counts = b.run()
            for i, s in enumerate(specs):
                n = s.shape[0]
                fop1, c1, hc1 = _single(plan, s)
                assert torch.equal(b.fop[i][:, :n], fop1[:, :n]), f"C={chunk} trial {i} (n={n}): FOP differs"
                _same(got[i], c1)
                assert np.array_equal(counts[i], hc1)
    finally:
        plan.destroy()


def test_autotune_keeps_results():
    plan = fdas.plan_create(n_max=1 << 17)
    other = None
    try:
        specs = _specs([40000, 100000, 70000, 9000], 61)
        b = Batch(plan, specs)
        t = fdas.autotune(plan, b.trials, repeats=2)
        print("autotune:", t, flush=True)
        assert 0 <= t["conv_templates_per_item"] <= 85 and t["conv_waves_per_simd"] in (1, 2)
        assert t["ols_chunk"] in (2048, 4096, 8192) and t["hsum_tile"] in (256, 512, 1024)
        got, _ = b.run()
        # the chosen chunk length computes the plane of a plan built for it
        ref = plan if t["ols_chunk"] == 4096 else fdas.plan_create(n_max=1 << 17, ols_chunk=t["ols_chunk"])
        other = ref if ref is not plan else None
        for i, s in enumerate(specs):
            _, c1, _ = _single(ref, s)
            _same(got[i], c1)
    finally:
        plan.destroy()
        if other is not None:
            other.destroy()


def test_batch_argument_errors():
    plan = plan42()
    L = fdas.lib()
    x = torch.zeros(100, dtype=torch.complex64, device=_dev())
    fop = torch.zeros((85, 128), dtype=torch.float32, device=_dev())
    cands, counts = fdas.alloc_cands(plan, _dev())
    good = fdas.trials_array([(x, 100, fop, 128, cands, counts)])
    assert L.fdas_search_batch(plan.handle, good, 0, None) == fdas.ERR_INVALID_ARG
    assert L.fdas_search_batch(plan.handle, None, 1, None) == fdas.ERR_INVALID_ARG
    bad = fdas.trials_array([(x, 100, fop, 99, cands, counts)])
    assert L.fdas_search_batch(plan.handle, bad, 1, None) == fdas.ERR_INVALID_ARG
    bad = fdas.trials_array([(x, 0, fop, 128, cands, counts)])
    assert L.fdas_search_batch(plan.handle, bad, 1, None) == fdas.ERR_INVALID_ARG
    t = fdas.Tuning()
    t.overlap_groups = 9
    assert L.fdas_set_tuning(plan.handle, t) == fdas.ERR_INVALID_ARG
    t = fdas.Tuning()
    t.ols_chunk = 1024
    assert L.fdas_set_tuning(plan.handle, t) == fdas.ERR_UNSUPPORTED
    t = fdas.Tuning()
    t.hsum_tile = 2048
    assert L.fdas_set_tuning(plan.handle, t) == fdas.ERR_UNSUPPORTED


def test_many_trials_in_one_readback():
    # 300 trials (the trial number needs more than 8 bits of the sort tag),
    # empty ones among them: every trial's list equals its single-call list
    plan = fdas.plan_create(n_max=1 << 14, cand_capacity=4096)
    try:
        base = _specs([1, 3000, 9000], 310)
        singles = [_single(plan, s) for s in base]
        specs = [base[i % 3] for i in range(300)]
        got, counts = Batch(plan, specs).run()
        for i in range(300):
            _, c1, hc1 = singles[i % 3]
            _same(got[i], c1)
            assert np.array_equal(counts[i], hc1)
    finally:
        plan.destroy()


def test_short_host_buffer_truncates_the_last_trials():
    plan = plan42()
    specs = _specs([40000, 3000, 65536], 320)
    b = Batch(plan, specs)
    full, _ = b.run()
    flat = np.concatenate(full)
    assert flat.size > 10
    short = flat.size - 7
    got, _ = fdas.candidates_batch(plan, b.trials, capacity=short, allow_overflow=True)
    _same(np.concatenate(got), flat[:short])
    L = fdas.lib()
    out = np.zeros(short, dtype=fdas.CAND_DTYPE)
    offs = np.zeros(len(specs) + 1, dtype=np.int64)
    st = L.fdas_candidates_batch(plan.handle, b.trials, len(specs), out.ctypes.data, short, offs.ctypes.data, None,
                                 None)
    assert st == fdas.ERR_CAPACITY
    assert offs[-1] == short and np.all(np.diff(offs) >= 0)
