"""FDAS hot-path benchmark on one MI355X.

One step = the whole hot path on one SKA-sized spectrum already resident in
HBM: fdas_convolve (85-template FT convolution + power -> FOP), then
fdas_harmonic_sum (8 harmonic planes, thresholds, candidate compaction), then
fdas_candidates (readback + canonical order).  Template generation happens
once at plan creation and is not timed.  Steps are pipelined (--pipeline,
default 2): step k+1's kernels are queued on a second plan and stream before
step k's candidates are ordered and copied back, so one spectrum's readback
and harmonic sum (HBM-bound) overlap the next one's convolution (ALU-bound),
as in a stream of dispersion trials; every step still does all of its work.
Kernel event times in the timed region then include the share of the chip
the other stream's kernels take; the same steps run one after the other are
reported beside them (serial_ms_per_step, roofline_isolated).

Prints one JSON line.  Per-kernel durations come from HIP events recorded on
the stream the library launches on; the roofline object describes the kernel
with the longest duration of its own (from the serial pass), timed in the
timed region.  The CPU baseline times the FP64 oracle
on a bounded sample (the first 2^20 bins of the same spectrum, median of three
runs on the threads this process may use) and scales it to spectra/s of the
full 2^22 workload by N log2 N.
"""

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FDAS spectra/s (2^22 pts, 85 templates, 8 harmonics) + % HBM/MFMA roofline"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, published
FP32_VECTOR_PEAK_TF = 157.3  # MI355X FP32 vector, published
FP32_MATRIX_PEAK_TF = 157.3  # MI355X FP32 matrix (dense), published
FP16_MATRIX_PEAK_TF = 2500.0  # MI355X FP16 / BF16 matrix (dense), published


# headers whose code is compiled into a kernel file's kernels
KERNEL_HEADERS = {"k_ols_conv.hip": ["fft16.h"]}


def kernel_source_digest(name):
    """sha256[:16] of a kernel source and of the headers its kernels inline."""
    h = hashlib.sha256()
    for f in [name] + KERNEL_HEADERS.get(name, []):
        with open(os.path.join(ROOT, "paper_1806_01556_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_file, launches_bytes_key):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or None.

    The summary carries a line `traffic: {json}` with the kernel source digest
    at the time the counters were taken; a different digest means stale
    counters, reported as null.
    """
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        for line in f:
            m = re.match(r"^traffic:\s*(\{.*\})\s*$", line.strip())
            if not m:
                continue
            rec = json.loads(m.group(1))
            if rec.get("kernel_file") != kernel_file:
                continue
            if rec.get("source_digest") != kernel_source_digest(kernel_file):
                return None
            return rec.get(launches_bytes_key)
    return None


def cpu_workers():
    """Threads this process may use: its scheduler CPU set, or fewer when
    OMP_NUM_THREADS names a smaller share of a shared machine."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, n_full, runs=3):
    """The FP64 oracle (FFT correlation with scipy.fft, then the harmonic sum
    and candidate list) on the first 2^20 bins of the spectrum, as one
    2^20-point spectrum, timed `runs` times; the median is scaled to the full
    length by N log2 N (the oracle's time is its 86 FFTs of about N points;
    the linear harmonic sum makes this scaling slightly pessimistic for the
    CPU)."""
    from oracle import fop as ofop
    from oracle import harmonic as oh

    n_s = min(1 << 20, spec.shape[0])
    workers = cpu_workers()
    x = spec[:n_s].astype(np.complex128)
    times, ncand = [], 0
    for _ in range(runs):
        t0 = time.perf_counter()
        plane = ofop.fop(x, workers=workers)
        cands = oh.candidates(plane, 8)
        times.append(time.perf_counter() - t0)
        ncand = int(cands.size)
        del plane
    dt = float(np.median(times))
    scale = (n_full * math.log2(n_full)) / (n_s * math.log2(n_s))
    return {
        "value": 1.0 / (dt * scale),
        "unit": "spectra/s",
        "cores": workers,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"first {n_s} bins of the same spectrum as one {n_s}-point spectrum (FP64 FFT correlation, "
                  f"{workers} scipy.fft threads, + harmonic sum, {ncand} candidates); median of {runs} runs "
                  f"{dt:.2f} s (runs {', '.join(f'{t:.2f}' for t in times)}), scaled to {n_full} bins by "
                  f"N log2 N = x{scale:.2f}",
    }


def bench_index_maps(args, torch, fdas, synth, dev):
    """Harmonic sum of one 2^22-bin plane (85 templates, 8 harmonics) under each
    index map: the stretch map of Algorithm 1 and the two alternatives built
    behind the plan option hsum_index.  One FOP (the overlap-save convolution
    of the headline spectrum) feeds all three; each call is timed with HIP
    events on the current stream, candidates included (counts reset, list
    appended), readback excluded."""
    n = 1 << 22
    spec, _ = synth.ska(n=n, seed=2)
    x = torch.from_numpy(spec).to(dev)
    maps = [("stretch", fdas.HSUM_STRETCH), ("fundamental", fdas.HSUM_FUNDAMENTAL),
            ("highest", fdas.HSUM_HIGHEST)]
    plans = {name: fdas.plan_create(n_max=n, hsum_index=idx) for name, idx in maps}
    fop = fdas.alloc_fop(plans["stretch"], n, dev)
    fdas.convolve(plans["stretch"], x, fop, n=n)
    torch.cuda.synchronize()
    plane_bytes = 85 * n * 4
    out = {"metric": "harmonic_sum_ms_per_plane", "unit": "ms", "higher_is_better": False, "data": "synthetic",
           "config": {"workload": "ska_single_spectrum_2^22 FOP, 85 templates, 8 harmonics, p_fa 1e-6"},
           "maps": {}}
    steps = max(1, args.steps)
    for name, _ in maps:
        plan = plans[name]
        cands, counts = fdas.alloc_cands(plan, dev)
        for _ in range(max(1, args.warmup)):
            fdas.harmonic_sum(plan, fop, n, cands, counts)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fdas.harmonic_sum(plan, fop, n, cands, counts)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        got, hc = fdas.candidates(plan, cands, counts, allow_overflow=True)
        out["maps"][name] = {"ms": round(ms, 4), "plane_reads_GB_per_s": round(plane_bytes / (ms * 1e-3) / 1e9, 1),
                             "candidates": int(got.size), "per_plane": [int(c) for c in hc]}
        print(f"index map {name}: {ms:.4f} ms per plane, {got.size} candidates", flush=True)
    for p in plans.values():
        p.destroy()
    print(json.dumps(out), flush=True)


def bench_batch(args, torch, fdas, synth, dev):
    """Batched dispersion trials: `trials` spectra of lengths drawn from
    {2^20, 2^21, 3*2^20, 2^22} (seeds 3000 + b, 0-4 pulsars each) per step,
    through fdas_search_batch + fdas_candidates_batch with the autotuned
    launch parameters; the same spectra through the single-spectrum calls
    are timed for comparison."""
    T = args.trials
    t_syn = time.perf_counter()
    specs = [synth.batch_member(b)[0] for b in range(T)]
    t_syn = time.perf_counter() - t_syn
    lens = [s.shape[0] for s in specs]
    n_max = max(lens)
    plan = fdas.plan_create(n_max=n_max)
    xs = [torch.from_numpy(s).to(dev) for s in specs]
    del specs
    fops = [torch.empty((plan.rows, fdas.fop_ld(n)), dtype=torch.float32, device=dev) for n in lens]
    bufs = [fdas.alloc_cands(plan, dev) for _ in lens]
    trials = fdas.trials_array([(x, n, f, f.shape[1], c[0], c[1]) for x, n, f, c in zip(xs, lens, fops, bufs)])
    stream = torch.cuda.current_stream()
    t_tune = time.perf_counter()
    tuning = fdas.autotune(plan, trials, repeats=2, stream=stream)
    t_tune = time.perf_counter() - t_tune

    def step():
        fdas.search_batch(plan, trials, stream=stream)
        return fdas.candidates_batch(plan, trials, stream=stream, allow_overflow=True, copy=False)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    gpu_ms = 0.0
    for _ in range(args.steps):
        e0.record(stream)
        fdas.search_batch(plan, trials, stream=stream)
        e1.record(stream)
        cands, counts = fdas.candidates_batch(plan, trials, stream=stream, allow_overflow=True, copy=False)
        gpu_ms += e0.elapsed_time(e1)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1e3 * wall / args.steps

    # the same trials one spectrum at a time through the single-spectrum calls
    single_steps = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(single_steps):
        for x, n, f, (c, k) in zip(xs, lens, fops, bufs):
            fdas.convolve(plan, x, f, n=n, stream=stream)
            fdas.harmonic_sum(plan, f, n, c, k, stream=stream)
            fdas.candidates(plan, c, k, stream=stream, allow_overflow=True, copy=False)
    torch.cuda.synchronize()
    single_ms = 1e3 * (time.perf_counter() - t1) / single_steps

    bins = int(sum(lens))
    hbm_bytes = 688 * bins                         # 8 + 340 B/bin conv, 340 B/bin harmonic sum
    out = {
        "metric": "FDAS spectra/s, batch of dispersion trials (uneven lengths, 85 templates, 8 harmonics)",
        "value": round(T * args.steps / wall, 3),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batch_{T}_trials", "trials": T, "lengths": sorted(set(lens)),
                   "total_bins": bins, "templates": 85, "harmonics": 8, "seeds": "3000+b",
                   "tuning": tuning},
        "chosen_ols_chunk": tuning["ols_chunk"],
        "chosen_hsum_tile_columns": tuning["hsum_tile"],
        "batch_gpu_ms_per_step": round(gpu_ms / args.steps, 3),
        "batch_hbm_gbs_algorithmic": round(hbm_bytes / (gpu_ms / args.steps * 1e-3) / 1e9, 1),
        "single_calls_ms_per_step": round(single_ms, 3),
        "single_calls_spectra_per_s": round(T / (single_ms * 1e-3), 3),
        "batch_speedup_vs_single_calls": round(single_ms / ms_per_step, 3),
        "candidates": int(sum(c.size for c in cands)),
        "setup_s": {"synthesis": round(t_syn, 1), "autotune": round(t_tune, 1)},
    }
    plan.destroy()
    print(json.dumps(out), flush=True)


PRESCREEN_TEST_SEED0 = 6_000_000


def _train_spectrum(args):
    """Training spectrum i of the label recipe (run in a worker process)."""
    return _val_spectrum(args)[0]


def _val_spectrum(args):
    """Labelled spectrum i of the label recipe with its pulsars (r, z, SNR,
    harmonics) (run in a worker process)."""
    from paper_1806_01556_amd import synth
    i, r = args
    spec, pulsars = synth.make_spectrum(r["n"], r["seed0"] + i, n_random=i % 4, r_range=tuple(r["r_range"]),
                                        z_range=tuple(r["z_range"]), snr_range=tuple(r["snr_range"]),
                                        harm_range=tuple(r["harm_range"]))
    return spec, [(p.r, p.z, p.snr, p.n_harm) for p in pulsars]


def _test_spectrum(i):
    """Test spectrum i: 2^22 bins, 1 + (i mod 3) pulsars with r ~ U[1e4, 2e6],
    z ~ U[-42, 42], SNR ~ U[5, 20], 1-8 harmonics (worker process)."""
    from paper_1806_01556_amd import synth
    spec, pulsars = synth.make_spectrum(1 << 22, PRESCREEN_TEST_SEED0 + i, n_random=1 + i % 3, r_range=(1e4, 2e6),
                                        snr_range=(5.0, 20.0))
    return spec, [(p.r, p.z, p.snr, p.n_harm) for p in pulsars]


def _spawn_map(fn, items, workers):
    """fn over items in fresh worker processes (spawned: the parent has a GPU
    context, which a forked child must not inherit), results in order."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, items, chunksize=max(1, len(items) // (4 * workers))))


def _keys(c):
    """int64 key (harm, z + 64, r) of each candidate record, sorted."""
    k = (c["harm"].astype(np.int64) << 40) | ((c["z"].astype(np.int64) + 64) << 32) | c["r"].astype(np.int64)
    return np.sort(k)


def _load_labels(name):
    """(recipe, [(i, block label string)]) of a pre-screen label fixture; rows
    stored as hex digits (block 0 in the leading bit) are expanded."""
    path = os.path.join(ROOT, "tests", "golden", name)
    with open(path) as f:
        lines = f.read().splitlines()
    recipe = json.loads(next(l for l in lines if l.startswith("# recipe: "))[len("# recipe: "):])
    nb = recipe["n"] // recipe["block"]
    rows = []
    for l in lines:
        if not l or l.startswith("#"):
            continue
        i, b = l.split()
        if len(b) != nb:
            b = format(int(b, 16), "0%db" % nb)
        rows.append((int(i), b))
    return recipe, rows


def bench_prescreen(args, torch, fdas, synth, dev):
    """Learned block pre-screen at the pre-screen workload's sizes: train on
    10,000 oracle-labelled spectra of 2^20 bins (tests/golden/
    prescreen_labels_2p20.txt, regenerated from their seeds; the 240 further
    labelled spectra pick the logit threshold), then search 256 spectra of
    2^22 bins on the flagged blocks and their harmonic multiples, against the
    plain search of the same spectra.  Recall is reported three ways: over
    every candidate cell of the plain search at the configured p_fa (1e-6),
    over its significant cells (power above T_k at a per-cell false-alarm
    probability of 1e-12, cells a screen can be asked to keep), and per
    injected pulsar the plain search detects."""
    label_file = "prescreen_labels_2p20.txt" if args.train_set == "2p20" else "prescreen_labels.txt"
    recipe, rows = _load_labels(label_file)
    nspec = len(rows)
    n_tr = recipe["n"]
    bpb = n_tr // 4096
    workers = cpu_workers()
    ps = fdas.Prescreen(max_batch=1024)  # one inference call covers a 2^22-bin spectrum
    # features of every block of every labelled spectrum stay on the device
    # (10,240 x 256 blocks x 16 KB = 43 GB at 2^20 bins); spectra are made by
    # worker processes in chunks and dropped once their features are formed
    feats = torch.empty((nspec * bpb, 4096), dtype=torch.float32, device=dev)
    labels = torch.tensor([float(c) for _, bits in rows for c in bits], dtype=torch.float32, device=dev)
    t_syn = time.perf_counter()
    chunk = 256
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        for c0 in range(0, nspec, chunk):
            part = rows[c0:c0 + chunk]
            specs = list(ex.map(_train_spectrum, [(i, recipe) for i, _ in part],
                                chunksize=max(1, len(part) // (2 * workers))))
            for k, sp in enumerate(specs):
                kk = c0 + k
                ps.features(torch.from_numpy(sp).to(dev), n_tr, bpb, feats[kk * bpb:(kk + 1) * bpb])
            del specs
            if (c0 // chunk) % 8 == 7:
                print(f"prescreen: {c0 + len(part)}/{nspec} training spectra made", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_syn = time.perf_counter() - t_syn
    n_train = min(args.train_spectra, nspec - 1)
    tr = np.arange(n_train * bpb)
    va = np.arange(n_train * bpb, nspec * bpb)
    lab_np = labels.cpu().numpy()
    pos = float(lab_np[tr].sum())
    pos_weight = (tr.size - pos) / max(pos, 1.0)
    ps.set_params(fdas.prescreen_init_params(0))
    rng = np.random.default_rng(0)  # batch order
    B = 256
    xb = torch.empty((B, 4096), dtype=torch.float32, device=dev)
    yb = torch.empty(B, dtype=torch.float32, device=dev)
    logit_b = torch.empty(B, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t_tr = time.perf_counter()
    steps, lr = 0, 2e-3
    for ep in range(args.epochs):
        perm = torch.from_numpy(rng.permutation(tr)).to(dev)
        for s0 in range(0, tr.size - B + 1, B):
            idx = perm[s0:s0 + B]
            torch.index_select(feats, 0, idx, out=xb)
            torch.index_select(labels, 0, idx, out=yb)
            ps.train_step(xb, yb, B, pos_weight, lr * (0.5 ** (ep // 4)), logit_b, loss)
            steps += 1
        print(f"prescreen: epoch {ep + 1}/{args.epochs}, batch loss {float(loss.item()):.4f}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t_tr
    final_loss = float(loss.item())

    def logits_of(fe, nb):
        out = torch.empty(nb, dtype=torch.float32, device=dev)
        for s0 in range(0, nb, ps.max_batch):
            m = min(ps.max_batch, nb - s0)
            ps.forward(fe[s0:s0 + m], m, out[s0:s0 + m])
        return out

    lv = logits_of(feats[va[0]:va[-1] + 1], va.size).cpu().numpy()
    yv = lab_np[va]
    del feats
    # operating points from the held-out data only.  The F2 point is the
    # logit threshold with the best F2 score (recall weighted four times
    # precision) on the held-out blocks, scanned over 1000 quantiles of their
    # logits; the val_qN points flag blocks above the N % quantile of the
    # held-out positive blocks' logits; the default, val_recall, is the
    # tightest threshold of a grid of such quantiles at which a search of the
    # held-out spectra keeps 0.999 of the significant cells of the plain
    # search there and the pulsars it detects with a one-sided 95 % lower
    # confidence bound (Clopper-Pearson) of at least 0.99 on the recall
    pos_v = yv > 0.5
    best = (-1.0, 0.0)
    for th in np.unique(np.quantile(lv, np.linspace(0.0, 1.0, 1001))):
        fl = lv > th
        tp = float(np.sum(fl & pos_v))
        rec, prec = tp / max(float(pos_v.sum()), 1.0), tp / max(float(fl.sum()), 1.0)
        f2 = 5.0 * prec * rec / max(4.0 * prec + rec, 1e-30)
        if f2 > best[0]:
            best = (f2, float(th))
    qs = [("val_f2", best[1])] + [(f"val_q{int(100 * q)}", float(np.quantile(lv[pos_v], q)))
                                  for q in (0.01, 0.02, 0.03, 0.05, 0.2, 0.5)]

    n = 1 << 22
    plan = fdas.plan_create(n_max=n)
    fop = fdas.alloc_fop(plan, n, dev)
    cands, counts = fdas.alloc_cands(plan, dev)
    tsig = fdas.thresholds(8, recipe["p_sig"]).astype(np.float32)
    rb_cap = plan.desc.n_harm * plan.desc.cand_capacity

    def significant(c):
        return c[c["power"] > tsig[c["harm"] - 1]]

    def evaluate(specs, puls, n_s, thresholds, progress=None):
        """Plain search vs the search of the flagged blocks (and their closure)
        of every spectrum, for every threshold: recall and block fractions."""
        nb = (n_s + 4095) // 4096
        lgt_s = torch.empty(nb, dtype=torch.float32, device=dev)
        st_all = {name: {"all": 0, "all_hit": 0, "sig": 0, "sig_hit": 0, "pul": 0, "pul_hit": 0, "flag": [],
                         "search": []} for name, _ in thresholds}
        ovf = 0
        for si, x in enumerate(specs):
            fdas.convolve(plan, x, fop, n=n_s)
            fdas.harmonic_sum(plan, fop, n_s, cands, counts)
            c_plain, hc = fdas.candidates(plan, cands, counts, capacity=rb_cap, allow_overflow=True)
            ovf += int(np.any(hc > plan.desc.cand_capacity))
            k_all, sig = _keys(c_plain), significant(c_plain)
            k_sig = _keys(sig)
            sig_blocks = set((sig["r"] // 4096).tolist())
            ps.infer(x, n_s, nb, lgt_s)
            lg = lgt_s.cpu().numpy()
            for name, th in thresholds:
                st = st_all[name]
                fdas.search_flagged(plan, x, n_s, fop, lgt_s, th, cands, counts)
                c_pre, _ = fdas.candidates(plan, cands, counts, capacity=rb_cap, allow_overflow=True)
                k_pre = _keys(c_pre)
                st["all"] += k_all.size
                st["all_hit"] += int(np.isin(k_all, k_pre, assume_unique=True).sum())
                st["sig"] += k_sig.size
                st["sig_hit"] += int(np.isin(k_sig, k_pre, assume_unique=True).sum())
                flagged = np.nonzero(lg > th)[0]
                st["flag"].append(flagged.size / nb)
                st["search"].append(fdas.block_closure(flagged, n_s).size / nb)
                got_blocks = set((c_pre["r"][c_pre["power"] > tsig[c_pre["harm"] - 1]] // 4096).tolist())
                for r0, _, _, _ in puls[si]:
                    b0 = int(r0) // 4096
                    near = {b0 - 1, b0, b0 + 1}
                    if near & sig_blocks:  # the plain search detects this pulsar
                        st["pul"] += 1
                        st["pul_hit"] += int(bool(near & sig_blocks & got_blocks))
            if progress and (si + 1) % 32 == 0:
                print(f"prescreen: {si + 1}/{len(specs)} {progress} spectra compared", file=sys.stderr, flush=True)
        return st_all, ovf

    def recall(st, key):
        return st[key + "_hit"] / max(st[key], 1)

    # the recall rule on held-out spectra of the label recipe: the first 240
    # after the training set (all of them at the default sizes)
    n_held = min(240, nspec - n_train)
    held = _spawn_map(_val_spectrum, [(i, recipe) for i, _ in rows[n_train:n_train + n_held]], workers)
    xs_val = [torch.from_numpy(sp).to(dev) for sp, _ in held]
    puls_val = [pl for _, pl in held]
    del held
    grid = [(f"g{k}", float(np.quantile(lv[pos_v], q))) for k, q in enumerate(np.linspace(0.005, 0.5, 40))]
    st_val, _ = evaluate(xs_val, puls_val, n_tr, grid, progress="held-out")
    from scipy.stats import beta

    def lower95(k, m):
        return float(beta.ppf(0.05, k, m - k + 1)) if k > 0 else 0.0

    ok_th = [(th, name) for name, th in grid
             if lower95(st_val[name]["pul_hit"], st_val[name]["pul"]) >= 0.99
             and recall(st_val[name], "sig") >= 0.999]
    th_rec = max(ok_th)[0] if ok_th else min(th for _, th in grid)
    rec_name = max(ok_th)[1] if ok_th else min(grid, key=lambda g: g[1])[0]
    val_rule = {"pulsars_detected_by_plain": st_val[rec_name]["pul"],
                "recall_pulsars": round(recall(st_val[rec_name], "pul"), 5),
                "recall_pulsars_lower95": round(lower95(st_val[rec_name]["pul_hit"], st_val[rec_name]["pul"]), 5),
                "recall_significant_cells": round(recall(st_val[rec_name], "sig"), 5),
                "searched_block_fraction": round(float(np.mean(st_val[rec_name]["search"])), 4)}
    del xs_val
    qs = [("val_recall", th_rec)] + qs
    val_flag = {name: round(float(np.mean(lv > th)), 4) for name, th in qs}
    val_recall = {name: round(float(np.mean(lv[yv > 0.5] > th)), 4) for name, th in qs}

    # ---- test spectra -------------------------------------------------------
    nblk = n // 4096
    T = args.test_spectra
    t_syn2 = time.perf_counter()
    test = _spawn_map(_test_spectrum, list(range(T)), workers)
    t_syn2 = time.perf_counter() - t_syn2
    xs = [torch.from_numpy(sp).to(dev) for sp, _ in test]
    pulsars = [pl for _, pl in test]
    del test
    stats, over = evaluate(xs, pulsars, n, qs, progress="test")

    # throughput with two spectra in flight, as in the headline: two plans,
    # pre-screens and streams; inference from the spectrum, device-side block
    # selection and search of spectrum k+1 are queued before the candidates of
    # spectrum k are read back (DMA), at the default threshold, against the
    # plain search run the same way, over the T test spectra
    thr = dict(qs)["val_recall"]
    theta = ps.get_params()
    pss = [ps, fdas.Prescreen(max_batch=1)]  # inference from the spectrum needs no batch workspace
    pss[1].set_params(theta)
    plans2 = [plan, fdas.plan_create(n_max=n)]
    fops2 = [fop, fdas.alloc_fop(plans2[1], n, dev)]
    bufs2 = [(cands, counts), fdas.alloc_cands(plans2[1], dev)]
    lgs = [torch.empty(nblk, dtype=torch.float32, device=dev) for _ in range(2)]
    strs = [torch.cuda.current_stream(), torch.cuda.Stream()]

    def pipe(steps, screened):
        for k in range(steps + 1):
            if k < steps:
                i, xk = k % 2, xs[k % T]
                st_ = strs[i]
                if screened:
                    pss[i].infer(xk, n, nblk, lgs[i], stream=st_)
                    fdas.search_flagged(plans2[i], xk, n, fops2[i], lgs[i], thr, bufs2[i][0], bufs2[i][1],
                                        stream=st_)
                else:
                    fdas.convolve(plans2[i], xk, fops2[i], n=n, stream=st_)
                    fdas.harmonic_sum(plans2[i], fops2[i], n, bufs2[i][0], bufs2[i][1], stream=st_)
            if k >= 1:
                j = (k - 1) % 2
                fdas.candidates(plans2[j], bufs2[j][0], bufs2[j][1], capacity=rb_cap, stream=strs[j],
                                allow_overflow=True, copy=False)

    pipe(4, True)
    pipe(4, False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pipe(T, True)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    t0 = time.perf_counter()
    pipe(T, False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    pss[1].destroy()
    plans2[1].destroy()

    points = {}
    for name, th in qs:
        st = stats[name]
        points[name] = {"logit_threshold": round(th, 4),
                        "recall_all_cells": round(st["all_hit"] / max(st["all"], 1), 5),
                        "recall_significant_cells": round(st["sig_hit"] / max(st["sig"], 1), 5),
                        "recall_pulsars": round(st["pul_hit"] / max(st["pul"], 1), 5),
                        "flagged_block_fraction": round(float(np.mean(st["flag"])), 4),
                        "searched_block_fraction": round(float(np.mean(st["search"])), 4),
                        "val_flagged_fraction": val_flag[name], "val_block_recall": val_recall[name]}
    head = points["val_recall"]
    st5 = stats["val_recall"]
    out = {
        "metric": "FDAS spectra/s with the learned block pre-screen (2^22 pts, 85 templates, 8 harmonics)",
        "value": round(T / t_pre, 3),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": T,
        "warmup": 4,
        "ms_per_step": round(1e3 * t_pre / T, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 search, bf16 network weights",
        "data": "synthetic",
        "config": {"workload": "prescreen_2^22", "test_spectra": T, "train_spectra": n_train,
                   "val_spectra": nspec - n_train, "val_search_spectra": n_held, "train_n": n_tr, "epochs": args.epochs, "train_steps": steps,
                   "pos_weight": round(pos_weight, 3), "p_fa": 1e-6, "p_label": recipe.get("p_label"),
                   "p_sig": recipe["p_sig"], "test_seeds": f"{PRESCREEN_TEST_SEED0}+i",
                   "train_label_file": label_file, "train_seeds": f"{recipe['seed0']}+i"},
        "plain_spectra_per_s": round(T / t_plain, 3),
        "speedup_vs_plain": round(t_plain / t_pre, 3),
        "recall_all_cells": head["recall_all_cells"],
        "recall_significant_cells": head["recall_significant_cells"],
        "recall_pulsars": head["recall_pulsars"],
        "plain_candidate_cells": st5["all"],
        "plain_significant_cells": st5["sig"],
        "pulsars_detected_by_plain": st5["pul"],
        "spectra_with_list_overflow": over,
        "operating_point": "val_recall: the tightest logit threshold at which a search of the 240 held-out "
                           "spectra keeps >= 0.999 of the significant cells of the plain search there and its "
                           "pulsars with a 95 % lower confidence bound >= 0.99; throughput with two spectra "
                           "in flight",
        "operating_point_held_out": val_rule,
        "operating_points": points,
        "train": {"final_batch_loss": round(final_loss, 5), "seconds": round(t_tr, 2),
                  "synthesis_s": round(t_syn, 1), "test_synthesis_s": round(t_syn2, 1), "workers": workers},
    }
    ps.destroy()
    plan.destroy()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--method", choices=("ols", "direct", "direct-fp16", "direct-bf16"), default="ols",
                    help="FT-convolution method: overlap-save FFT (default, the faster) or the direct "
                         "correlation on the matrix cores")
    ap.add_argument("--readback", choices=["auto", "mapped", "copy"], default="auto",
                    help="candidate readback: fdas_candidates_mapped (a kernel writes to pinned memory, one "
                         "wait) or fdas_candidates (DMA copy, two waits); auto = copy with steps in flight "
                         "(no compute units held by PCIe writes beside the next step's kernels), mapped "
                         "otherwise")
    ap.add_argument("--ols-chunk", type=int, default=0, choices=(0, 2048, 4096, 8192),
                    help="overlap-save chunk length C of the plans (0 = the library default, 4096)")
    ap.add_argument("--emit-workgroups", type=int, default=0,
                    help="workgroups of the harmonic sum's candidate emission (64..16384; 0 = the library default)")
    ap.add_argument("--step-order", choices=("overlap", "chain", "staged", "hs-chain"), default="overlap",
                    help="with steps in flight: overlap = the kernels of the two streams share the chip; chain = a "
                         "step's convolution waits on the device for the previous step's harmonic sum; staged = "
                         "chain, and the previous step's ordering and readback also wait for this step's "
                         "convolution (they run beside its harmonic sum); hs-chain = only a step's harmonic sum "
                         "waits for the previous one")
    ap.add_argument("--pipeline", type=int, default=2,
                    help="steps in flight in the timed region: with 2 (default), step k+1's kernels are "
                         "queued on a second plan and stream before step k's candidates are read back; "
                         "1 runs one step after the other")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="label the FOP-buffer copies made after timing (4 plain copies of known size, "
                         "also timed as the achievable HBM bandwidth) so HBM counters can be scaled to bytes")
    ap.add_argument("--workload", choices=("ska", "batch", "prescreen", "index-maps"), default="ska",
                    help="ska: one 2^22-bin spectrum per step (the headline); batch: 64 dispersion trials of "
                         "uneven length per step through the batch calls; prescreen: train the learned block "
                         "pre-screen on oracle-labelled spectra, then search 2^22-bin spectra on flagged blocks; "
                         "index-maps: the harmonic sum of one 2^22-bin plane under each index map")
    ap.add_argument("--epochs", type=int, default=8, help="prescreen workload: training epochs")
    ap.add_argument("--train-set", choices=("2p20", "2p16"), default="2p20",
                    help="prescreen workload: labelled spectra of 2^20 bins (tests/golden/prescreen_labels_2p20.txt, "
                         "default) or of 2^16 bins (tests/golden/prescreen_labels.txt)")
    ap.add_argument("--train-spectra", type=int, default=10000,
                    help="prescreen workload: labelled spectra to train on (the rest pick the threshold)")
    ap.add_argument("--test-spectra", type=int, default=256, help="prescreen workload: 2^22-bin test spectra")
    ap.add_argument("--trials", type=int, default=64, help="batch workload: trials per step")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(spectra are independent, so several GPUs would each run this same workload)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1806_01556_amd import fdas, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    fdas.lib()  # raises if libfdas.so is missing
    if args.workload == "batch":
        return bench_batch(args, torch, fdas, synth, dev)
    if args.workload == "prescreen":
        return bench_prescreen(args, torch, fdas, synth, dev)
    if args.workload == "index-maps":
        return bench_index_maps(args, torch, fdas, synth, dev)

    n = 1 << 22
    spec, pulsars = synth.ska(n=n, seed=2)
    x = torch.from_numpy(spec).to(dev)
    method = fdas.CONV_OLS_FFT if args.method == "ols" else fdas.CONV_DIRECT_MFMA
    precision = {"direct-fp16": fdas.PREC_SPLIT_FP16, "direct-bf16": fdas.PREC_SPLIT_BF16}.get(args.method,
                                                                                             fdas.PREC_FP32)
    P = max(1, args.pipeline)
    NP = max(P, 2)
    # NP independent plans, FOPs, candidate buffers and streams: with P steps
    # in flight step k uses set k % P, so step k's kernels run while step
    # k-1's candidates are ordered and copied back (a plan is used by one
    # stream at a time)
    C = args.ols_chunk or 4096
    plans = [fdas.plan_create(n_max=n, method=method, precision=precision, ols_chunk=C) for _ in range(NP)]
    if args.emit_workgroups:
        for p_ in plans:
            fdas.set_tuning(p_, emit_workgroups=args.emit_workgroups)
    fops = [fdas.alloc_fop(plans[i], n, dev) for i in range(NP)]
    bufs = [fdas.alloc_cands(plans[i], dev) for i in range(NP)]
    streams = [torch.cuda.current_stream()] + [torch.cuda.Stream() for _ in range(NP - 1)]

    # --step-order: "overlap" leaves the two streams' kernels to share the
    # chip; "chain" makes step k's convolution wait (on the device) for step
    # k-1's harmonic sum, so only the ordering and readback of a step overlap
    # the next step's kernels; "staged" also makes the ordering of step k-1
    # wait for step k's convolution, so the convolution runs alone and the
    # ordering runs beside the harmonic sum; "hs-chain" only keeps two
    # harmonic sums from running at once
    hs_done = [torch.cuda.Event() for _ in range(NP)]
    conv_done = [torch.cuda.Event() for _ in range(NP)]

    def enqueue(k, ev=None, P=P):
        i = k % P
        st = streams[i]
        if args.step_order in ("chain", "staged") and P > 1 and k > 0:
            st.wait_event(hs_done[(k - 1) % P])
        if ev:
            ev[0].record(st)
        fdas.convolve(plans[i], x, fops[i], n=n, stream=st)
        conv_done[i].record(st)
        if ev:
            ev[1].record(st)
        if args.step_order == "hs-chain" and P > 1 and k > 0:
            st.wait_event(hs_done[(k - 1) % P])
        fdas.harmonic_sum(plans[i], fops[i], n, bufs[i][0], bufs[i][1], stream=st)
        hs_done[i].record(st)
        if ev:
            ev[2].record(st)

    # mapped: the ordered records are written into page-locked host memory by
    # a kernel (one wait); copy: a DMA copy after a wait for the counts (two
    # waits, no compute units busy with PCIe writes)
    if args.readback == "auto":
        args.readback = "copy" if P > 1 else "mapped"
    rb_cap = None if args.readback == "mapped" else plans[0].desc.n_harm * plans[0].desc.cand_capacity

    def readback(k, P=P):
        i = k % P
        return fdas.candidates(plans[i], bufs[i][0], bufs[i][1], capacity=rb_cap, stream=streams[i],
                               allow_overflow=True, copy=False)

    def run(steps, evs=None, P=P):
        out = None
        for k in range(steps):
            enqueue(k, evs[k] if evs else None, P)
            if k >= P - 1:
                if args.step_order == "staged" and P > 1:
                    streams[(k - P + 1) % P].wait_event(conv_done[k % P])
                out = readback(k - P + 1, P)
        for k in range(max(0, steps - P + 1), steps):
            out = readback(k, P)
        return out

    run(args.warmup)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    c, hc = run(args.steps, evs)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ncand = int(c.size)

    conv_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    hs_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    ms_per_step = 1e3 * wall / args.steps

    # the same steps one after another on one stream (no overlap), for reference
    serial_steps = min(args.steps, 10)
    sevs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(serial_steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for k in range(serial_steps):
        enqueue(0, sevs[k])
        readback(0)
    torch.cuda.synchronize()
    serial_ms = 1e3 * (time.perf_counter() - t1) / serial_steps
    conv_ms_serial = float(np.mean([e[0].elapsed_time(e[1]) for e in sevs]))
    hs_ms_serial = float(np.mean([e[1].elapsed_time(e[2]) for e in sevs]))

    # the candidate readback alone (ordering on the device + copy of the
    # records to the host), after the harmonic sum has finished
    rb_ms = []
    for k in range(5):
        enqueue(0)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        readback(0)
        rb_ms.append(1e3 * (time.perf_counter() - t3))

    # two steps in flight (two plans and streams), untimed per kernel
    pipe = None
    if P == 1:
        run(2, None, 2)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        run(args.steps, None, 2)
        torch.cuda.synchronize()
        w2 = time.perf_counter() - t2
        pipe = {"spectra_per_s": round(args.steps / w2, 3), "ms_per_step": round(1e3 * w2 / args.steps, 4),
                "note": "two plans on two streams: one spectrum's readback and harmonic sum overlap the "
                        "next one's convolution"}

    V = C - 393                                      # valid outputs per C-point chunk
    hs_bytes = 4 * 85 * n                            # FOP read once
    conv_bytes = 8 * n + 4 * 85 * n                  # spectrum read + FOP write
    if args.method == "ols":
        conv_flop = 85 * 5 * C * math.log2(C) / V * n  # algorithmic FFT flops of one launch
        conv = {"name": "k_ols_conv", "bound": "alu", "peak": FP32_VECTOR_PEAK_TF, "file": "k_ols_conv.hip"}
    elif args.method == "direct":
        taps = sum(2 * (8 + (9 * abs(z) + 1) // 2) for z in range(-42, 43))
        conv_flop = 8 * taps * n                     # one complex multiply-add per template tap and bin
        conv = {"name": "k_direct_conv", "bound": "mfma", "peak": FP32_MATRIX_PEAK_TF,
                "file": "k_direct_conv.hip"}
    else:
        # split precision: three 16-bit products per FP32 product; the
        # contraction's useful flops counted once, against the 16-bit peak
        taps = sum(2 * (8 + (9 * abs(z) + 1) // 2) for z in range(-42, 43))
        conv_flop = 8 * taps * n
        conv = {"name": "k_direct_conv_split", "bound": "mfma", "peak": FP16_MATRIX_PEAK_TF,
                "file": "k_direct_conv.hip"}
    kernels = {
        conv["name"]: {"ms": conv_ms, "bound": conv["bound"], "achieved": conv_flop / (conv_ms * 1e-3) / 1e12,
                       "peak": conv["peak"], "unit": "TFLOP/s", "file": conv["file"],
                       "hbm_gbs": conv_bytes / (conv_ms * 1e-3) / 1e9},
        "k_harmsum": {"ms": hs_ms, "bound": "hbm", "achieved": hs_bytes / (hs_ms * 1e-3) / 1e9,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "file": "k_harmsum.hip"},
    }
    # the dominant kernel is the one with the longer time of its own (serial
    # pass); with two steps in flight the timed-region durations of the two
    # kernels include each other's share of the chip and can swap order
    own_ms = {conv["name"]: conv_ms_serial, "k_harmsum": hs_ms_serial}
    dom_name = max(kernels, key=lambda k: own_ms[k])
    dom = kernels[dom_name]
    roof = {
        "kernel": dom_name,
        "bound": dom["bound"],
        "achieved": round(dom["achieved"], 3),
        "peak": dom["peak"],
        "unit": dom["unit"],
        "frac": round(dom["achieved"] / dom["peak"], 4),
        # the counters were taken at the default chunk length
        "traffic": read_traffic(dom["file"], "bytes_per_launch") if C == 4096 or dom_name != "k_ols_conv" else None,
    }
    # the same kernel timed in the serial pass (no other step's kernels beside it)
    conv_work = conv_flop / 1e12
    iso_ms = conv_ms_serial if dom_name == conv["name"] else hs_ms_serial
    iso_ach = (conv_work / (iso_ms * 1e-3)) if dom_name == conv["name"] else hs_bytes / (iso_ms * 1e-3) / 1e9
    roof_iso = {"kernel": dom_name, "avg_ms": round(iso_ms, 4), "achieved": round(iso_ach, 3),
                "peak": dom["peak"], "unit": dom["unit"], "frac": round(iso_ach / dom["peak"], 4),
                "note": "serial pass; the headline roofline times the kernel while the other step's "
                        "kernels may share the GPU"}

    if args.method in ("direct-fp16", "direct-bf16"):
        # matrix-core work the split kernel issues: its 11 template tiles
        # (85 templates by |z|, 8 per tile, each over the union of its
        # members' supports padded to 8 tap pairs) make 163 groups of 16 taps
        # per 16 bins, each 3 v_mfma_f32_16x16x32 of 16,384 flop
        issued = 163 * 3 * 16384 / 16 * n
        issued_tf = issued / (conv_ms * 1e-3) / 1e12
        roof["mfma_issued"] = {"achieved": round(issued_tf, 3), "peak": FP16_MATRIX_PEAK_TF, "unit": "TFLOP/s",
                               "frac": round(issued_tf / FP16_MATRIX_PEAK_TF, 4),
                               "note": "hi*hi + hi*lo + lo*hi products and padded taps included"}
    out = {
        "metric": METRIC,
        "value": round(args.steps / wall, 3),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "ska_single_spectrum_2^22", "n": n, "templates": 85, "z_max": 42,
                   "harmonics": 8, "p_fa": 1e-6, "pulsars": len(pulsars), "seed": 2,
                   "method": {"ols": f"ols_fft_c{C}", "direct": "direct_mfma_fp32",
                              "direct-fp16": "direct_mfma_split_fp16",
                              "direct-bf16": "direct_mfma_split_bf16"}[args.method],
                   "pipeline": P, "readback": args.readback, "step_order": args.step_order,
                   "emit_workgroups": args.emit_workgroups or 1024},
        "roofline": roof,
        "roofline_isolated": roof_iso,
        "stages_ms": {"convolve": round(conv_ms, 4), "harmonic_sum": round(hs_ms, 4),
                      "note": "event times in the timed region, where two steps are in flight and each "
                              "kernel shares the GPU with the other step's work"},
        "stages_median_ms": {"convolve": round(float(np.median([e[0].elapsed_time(e[1]) for e in evs])), 4),
                             "harmonic_sum": round(float(np.median([e[1].elapsed_time(e[2]) for e in evs])), 4)},
        "serial_ms_per_step": round(serial_ms, 4),
        "readback_ms": {"median": round(float(np.median(rb_ms)), 4), "readback": args.readback,
                        "note": "candidate ordering on the device and copy to the host, timed alone after the "
                                "harmonic sum (inside every step above)"},
        "pipelined_2": pipe,
        "serial_stages_ms": {"convolve": round(conv_ms_serial, 4), "harmonic_sum": round(hs_ms_serial, 4)},
        "kernels": {k: {"avg_ms": round(v["ms"], 4), "achieved": round(v["achieved"], 3), "unit": v["unit"],
                        "frac": round(v["achieved"] / v["peak"], 4)} for k, v in kernels.items()},
        "conv_hbm_gbs": round(kernels[conv["name"]]["hbm_gbs"], 1),
        "candidates": ncand,
        "candidates_per_plane": [int(v) for v in hc],
    }
    # achievable HBM bandwidth beside the 8 TB/s spec: a plain device copy of
    # the FOP buffer (read + write), after the timed region; with
    # --calibrate-copy the same copies scale the HBM counters
    src = fops[0].view(-1)
    dst = torch.empty_like(src)
    ce = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    dst.copy_(src)
    ce[0].record()
    for _ in range(3):
        dst.copy_(src)
    ce[1].record()
    torch.cuda.synchronize()
    copy_ms = ce[0].elapsed_time(ce[1]) / 3
    out["hbm_copy"] = {"bytes": 2 * src.numel() * 4, "ms": round(copy_ms, 4),
                       "gbs": round(2 * src.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1)}
    if args.calibrate_copy:
        out["calibration_copy_bytes"] = {"read": src.numel() * 4, "write": src.numel() * 4}
    del dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, n)
    for pl in plans:
        pl.destroy()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
