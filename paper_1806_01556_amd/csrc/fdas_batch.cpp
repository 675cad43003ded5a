// Batch calls of the C ABI: many dispersion-trial spectra of uneven length in
// one persistent convolution launch and one harmonic-sum launch per overlap
// group, recorded once as a HIP graph and replayed (fdas_search_batch); one
// readback for all trials (fdas_candidates_batch); a measured choice of the
// launch parameters (fdas_autotune).
//
// Graph layout for G overlap groups (trials split into G contiguous groups of
// about equal length):
//   capture stream: zero counts -> conv(group 0) -> conv(group 1) -> ...
//   side stream:                    \-> hsum(group 0) \-> hsum(group 1) ...
// so the memory-bound harmonic sum of one group runs while the arithmetic-
// bound convolution of the next group occupies the compute units (the
// pipeline computing of Section 3.3; every trial has its own FOP buffer).
// The graph reads its per-trial parameters from plan-owned device tables that
// are refreshed before every launch, so it is recorded again only when the
// launch shape changes.

#include <algorithm>
#include <cstring>
#include <vector>

#include "fdas_plan.h"

namespace fdas {

void free_batch(fdas_plan* p) {
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  p->graph_exec = nullptr;
  if (p->graph_done) (void)hipEventDestroy(p->graph_done);
  for (hipEvent_t e : p->fork_events) (void)hipEventDestroy(e);
  p->fork_events.clear();
  if (p->stage_done) (void)hipEventDestroy(p->stage_done);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->side_stream) (void)hipStreamDestroy(p->side_stream);
  if (p->d_conv_trials) (void)hipFree(p->d_conv_trials);
  if (p->d_hs_trials) (void)hipFree(p->d_hs_trials);
  if (p->h_stage) (void)hipHostFree(p->h_stage);
  if (p->d_bhitrows) (void)hipFree(p->d_bhitrows);
  if (p->d_bhitrow_count) (void)hipFree(p->d_bhitrow_count);
  if (p->d_cand_ptrs) (void)hipFree(p->d_cand_ptrs);
  if (p->d_counts_all) (void)hipFree(p->d_counts_all);
  if (p->h_counts_all) (void)hipHostFree(p->h_counts_all);
  if (p->d_rb_tab) (void)hipFree(p->d_rb_tab);
  if (p->d_bsort_a) (void)hipFree(p->d_bsort_a);
  if (p->d_bsort_b) (void)hipFree(p->d_bsort_b);
  if (p->d_bsort_hist) (void)hipFree(p->d_bsort_hist);
  if (p->d_bsort_totals) (void)hipFree(p->d_bsort_totals);
}

}  // namespace fdas

using namespace fdas;

namespace {

constexpr int kMaxTrials = 1024;
constexpr int kMaxGroups = 8;

fdas_status check_trials(const fdas_plan* p, const fdas_trial* t, int count, bool need_fop) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!t) return fail(FDAS_ERR_INVALID_ARG, "trial array is NULL");
  if (count < 1 || count > kMaxTrials) return fail(FDAS_ERR_INVALID_ARG, "count = %d outside [1, %d]", count, kMaxTrials);
  for (int i = 0; i < count; ++i) {
    if (need_fop) {
      if (!t[i].d_spectrum) return fail(FDAS_ERR_INVALID_ARG, "trial %d: spectrum pointer is NULL", i);
      if (reinterpret_cast<uintptr_t>(t[i].d_spectrum) % 8 != 0)
        return fail(FDAS_ERR_INVALID_ARG, "trial %d: spectrum pointer must be 8-byte aligned", i);
      fdas_status st = check_fop_args(p, t[i].d_fop, t[i].n, t[i].ld);
      if (st != FDAS_OK) return fail(st, "trial %d: %s", i, fdas_last_error());
    }
    if (!t[i].d_cands || reinterpret_cast<uintptr_t>(t[i].d_cands) % 16 != 0)
      return fail(FDAS_ERR_INVALID_ARG, "trial %d: candidate buffer is NULL or not 16-byte aligned", i);
    if (!t[i].d_counts || reinterpret_cast<uintptr_t>(t[i].d_counts) % 4 != 0)
      return fail(FDAS_ERR_INVALID_ARG, "trial %d: count buffer is NULL or misaligned", i);
  }
  return FDAS_OK;
}

void invalidate_graph(fdas_plan* p) {
  // a graph still in flight keeps using the tables: wait for its last launch
  if (p->graph_exec && p->graph_done) (void)hipEventSynchronize(p->graph_done);
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  p->graph_exec = nullptr;
  p->graph_key.clear();
}

hipError_t ensure_streams(fdas_plan* p) {
  hipError_t e = hipSuccess;
  if (!p->cap_stream && (e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  if (!p->side_stream && (e = hipStreamCreateWithFlags(&p->side_stream, hipStreamNonBlocking)) != hipSuccess) return e;
  if (!p->stage_done && (e = hipEventCreateWithFlags(&p->stage_done, hipEventDisableTiming)) != hipSuccess) return e;
  if (!p->graph_done && (e = hipEventCreateWithFlags(&p->graph_done, hipEventDisableTiming)) != hipSuccess) return e;
  while ((int)p->fork_events.size() < kMaxGroups + 1) {
    hipEvent_t ev = nullptr;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) return e;
    p->fork_events.push_back(ev);
  }
  return hipSuccess;
}

// tables for `count` trials and a pinned staging area of `stage_bytes`
hipError_t ensure_tables(fdas_plan* p, int count, size_t stage_bytes) {
  hipError_t e = hipSuccess;
  if (count > p->batch_cap) {
    invalidate_graph(p);
    if (p->d_conv_trials) (void)hipFree(p->d_conv_trials);
    if (p->d_hs_trials) (void)hipFree(p->d_hs_trials);
    p->d_conv_trials = nullptr;
    p->d_hs_trials = nullptr;
    p->batch_cap = 0;
    const int cap = std::max(count, 64);
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_conv_trials), cap * sizeof(ConvTrial))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_hs_trials), cap * sizeof(HsTrial))) != hipSuccess) return e;
    p->batch_cap = cap;
  }
  if (stage_bytes > p->h_stage_bytes) {
    if (p->h_stage) {
      // the previous upload from the staging area must have been consumed
      if (p->stage_done) (void)hipEventSynchronize(p->stage_done);
      (void)hipHostFree(p->h_stage);
    }
    p->h_stage = nullptr;
    p->h_stage_bytes = 0;
    if ((e = hipHostMalloc(&p->h_stage, stage_bytes, 0)) != hipSuccess) return e;
    p->h_stage_bytes = stage_bytes;
  }
  return hipSuccess;
}

struct Launch {
  const OlsTables* ols = nullptr;          // chunk length of the convolution
  int tpg = 0, slots = 0, groups = 1, eblocks = 1024, cols = 1024;
  std::vector<int> tlo, thi;               // trials of each group
  std::vector<int64_t> ilo, ihi;           // convolution items of each group
  std::vector<int> blo, bhi;               // harmonic-sum workgroups of each group
  int64_t hitrows_needed = 0;              // largest hit-row list of a group
};

// Per-trial table entries and the group split.
fdas_status plan_launch(fdas_plan* p, const fdas_trial* t, int count, Launch& L, ConvTrial* ct, HsTrial* ht) {
  const int rows = p->rows;
  const int C = p->tuning.ols_chunk > 0 ? p->tuning.ols_chunk : p->ols[p->ols_idx].geom.C;
  hipError_t e0 = ols_tables(p, C, &L.ols);
  if (e0 != hipSuccess) return hip_fail(e0, "building the overlap-save tables of the batch's chunk length");
  const int V = L.ols->geom.V;
  // waves per SIMD -> workgroups per compute unit (4 SIMDs, C/16 threads per workgroup)
  const int wps = p->tuning.conv_waves_per_simd > 0 ? p->tuning.conv_waves_per_simd : 2;
  L.slots = p->cus * std::max(1, 4 * wps * 64 / ols_threads(C));
  L.cols = p->tuning.hsum_tile > 0 ? p->tuning.hsum_tile : 1024;
  // 0: every workgroup's range of (chunk, template) pairs shares one forward
  // FFT per chunk it touches
  L.tpg = p->tuning.conv_templates_per_item > 0 ? std::min(rows, p->tuning.conv_templates_per_item) : 0;
  L.eblocks = p->tuning.emit_workgroups > 0 ? p->tuning.emit_workgroups : 1024;
  int64_t item = 0;
  int block = 0;
  for (int i = 0; i < count; ++i) {
    const int* order = nullptr;
    int nblocks = 0;
    hipError_t e = tile_order_for(p, t[i].n, &order, &nblocks, L.cols);
    if (e != hipSuccess) return hip_fail(e, "uploading a harmonic-sum tile order");
    ct[i] = ConvTrial{static_cast<const float2*>(t[i].d_spectrum), t[i].d_fop, t[i].n, t[i].ld, item};
    ht[i] = HsTrial{t[i].d_fop, t[i].ld, t[i].d_cands, t[i].d_counts, order, (int)t[i].n, block, nblocks, 0};
    item += ((t[i].n + V - 1) / V) * rows;
    block += nblocks;  // a multiple of 8: every trial starts on XCD 0
  }
  // contiguous groups of about equal total length
  int64_t total = 0;
  for (int i = 0; i < count; ++i) total += t[i].n;
  const int G = std::max(1, std::min({p->tuning.overlap_groups > 0 ? p->tuning.overlap_groups : 1, count, kMaxGroups}));
  L.groups = 0;
  L.tlo.clear(); L.thi.clear(); L.ilo.clear(); L.ihi.clear(); L.blo.clear(); L.bhi.clear();
  L.hitrows_needed = 1;
  int lo = 0;
  int64_t acc = 0;
  for (int g = 0; g < G && lo < count; ++g) {
    int hi = lo;
    const int64_t target = total * (g + 1) / G;
    do {
      acc += t[hi].n;
      ++hi;
    } while (hi < count && acc < target && count - hi > G - g - 1);
    if (g == G - 1) {
      while (hi < count) acc += t[hi++].n;
    }
    L.tlo.push_back(lo);
    L.thi.push_back(hi);
    L.ilo.push_back(ct[lo].item0);
    L.ihi.push_back(hi < count ? ct[hi].item0 : item);
    L.blo.push_back(ht[lo].block0);
    L.bhi.push_back(hi < count ? ht[hi].block0 : block);
    int64_t hr = 0;
    for (int i = lo; i < hi; ++i) hr += (t[i].n + 3) / 4;
    L.hitrows_needed = std::max(L.hitrows_needed, hr);
    ++L.groups;
    lo = hi;
  }
  return FDAS_OK;
}

hipError_t record_sequence(fdas_plan* p, int count, const Launch& L) {
  hipStream_t cs = p->cap_stream, ss = p->side_stream;
  hipError_t e = launch_zero_counts_batch(p->d_hs_trials, count, p->desc.n_harm, cs);
  for (int g = 0; g < L.groups && e == hipSuccess; ++g) {
    e = launch_ols_conv_batch(p->d_conv_trials, count, L.ilo[g], L.ihi[g], *L.ols, p->rows, L.tpg, L.slots, cs);
    if (e == hipSuccess) e = hipEventRecord(p->fork_events[g], cs);
    if (e == hipSuccess) e = hipStreamWaitEvent(ss, p->fork_events[g], 0);
    if (e == hipSuccess)
      e = launch_harmsum_batch85(p->d_hs_trials, count, L.blo[g], L.bhi[g], p->desc.n_harm, p->d_ta,
                                 p->desc.cand_capacity, p->d_bhitrows, p->d_bhitrow_count, L.eblocks, L.cols, ss);
  }
  if (e == hipSuccess) e = hipEventRecord(p->fork_events[kMaxGroups], ss);
  if (e == hipSuccess) e = hipStreamWaitEvent(cs, p->fork_events[kMaxGroups], 0);
  return e;
}

// The graphed path: overlap-save convolution and the two-phase 85-row stretch sum.
bool graphable(const fdas_plan* p) {
  return !p->direct && p->desc.z_max == 42 && p->desc.hsum_index == FDAS_HSUM_STRETCH;
}

fdas_status search_batch(fdas_plan* p, const fdas_trial* t, int count, hipStream_t s) {
  if (!graphable(p)) {
    // other methods and index maps: the single-spectrum calls in turn
    for (int i = 0; i < count; ++i) {
      fdas_status st = fdas_convolve(p, t[i].d_spectrum, t[i].n, t[i].d_fop, t[i].ld, s);
      if (st == FDAS_OK) st = fdas_harmonic_sum(p, t[i].d_fop, t[i].n, t[i].ld, nullptr, t[i].d_cands, t[i].d_counts, s);
      if (st != FDAS_OK) return st;
    }
    return ok();
  }
  hipError_t e = ensure_streams(p);
  if (e != hipSuccess) return hip_fail(e, "creating the batch streams");
  const size_t stage_bytes = (size_t)count * (sizeof(ConvTrial) + sizeof(HsTrial));
  // the staging area may still feed the previous call's upload
  if (p->stage_done && p->h_stage) (void)hipEventSynchronize(p->stage_done);
  e = ensure_tables(p, count, stage_bytes);
  if (e != hipSuccess) return hip_fail(e, "allocating the batch tables");
  ConvTrial* ct = static_cast<ConvTrial*>(p->h_stage);
  HsTrial* ht = reinterpret_cast<HsTrial*>(static_cast<char*>(p->h_stage) + (size_t)count * sizeof(ConvTrial));
  Launch L;
  fdas_status st = plan_launch(p, t, count, L, ct, ht);
  if (st != FDAS_OK) return st;
  if (L.hitrows_needed > p->bhitrows_cap) {
    invalidate_graph(p);
    if (p->d_bhitrows) (void)hipFree(p->d_bhitrows);
    p->d_bhitrows = nullptr;
    p->bhitrows_cap = 0;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_bhitrows), L.hitrows_needed * sizeof(int4))) != hipSuccess)
      return hip_fail(e, "allocating the batch hit-row list");
    p->bhitrows_cap = L.hitrows_needed;
  }
  if (!p->d_bhitrow_count && (e = hipMalloc(reinterpret_cast<void**>(&p->d_bhitrow_count), sizeof(int32_t))) != hipSuccess)
    return hip_fail(e, "allocating the batch hit-row counter");
  // refresh the device tables (ordered before the graph on the caller's stream)
  if ((e = hipMemcpyAsync(p->d_conv_trials, ct, count * sizeof(ConvTrial), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(p->d_hs_trials, ht, count * sizeof(HsTrial), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipEventRecord(p->stage_done, s)) != hipSuccess)
    return hip_fail(e, "uploading the batch tables");
  std::vector<int64_t> key = {count, L.tpg, L.slots, L.groups, L.eblocks, p->desc.n_harm, L.ols->geom.C, L.cols,
                              (int64_t)(uintptr_t)p->d_conv_trials, (int64_t)(uintptr_t)p->d_hs_trials,
                              (int64_t)(uintptr_t)p->d_bhitrows};
  for (int g = 0; g < L.groups; ++g) {
    key.push_back(L.ilo[g]);
    key.push_back(L.ihi[g]);
    key.push_back(L.blo[g]);
    key.push_back(L.bhi[g]);
  }
  if (!p->graph_exec || key != p->graph_key) {
    invalidate_graph(p);
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "starting the batch graph capture");
    hipError_t er = record_sequence(p, count, L);
    e = hipStreamEndCapture(p->cap_stream, &graph);
    if (er != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return hip_fail(er, "recording the batch graph");
    }
    if (e != hipSuccess) return hip_fail(e, "ending the batch graph capture");
    e = hipGraphInstantiate(&p->graph_exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      p->graph_exec = nullptr;
      return hip_fail(e, "instantiating the batch graph");
    }
    p->graph_key = key;
  }
  e = hipGraphLaunch(p->graph_exec, s);
  if (e == hipSuccess) e = hipEventRecord(p->graph_done, s);
  if (e != hipSuccess) return hip_fail(e, "launching the batch graph");
  return ok();
}

}  // namespace

extern "C" {

fdas_status fdas_search_batch(fdas_plan* p, const fdas_trial* h_trials, int32_t count, void* stream) {
  fdas_status st = check_trials(p, h_trials, count, true);
  if (st != FDAS_OK) return st;
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  return search_batch(p, h_trials, count, static_cast<hipStream_t>(stream));
}

fdas_status fdas_candidates_batch(fdas_plan* p, const fdas_trial* h_trials, int32_t count, fdas_cand* h_out,
                                  int64_t h_capacity, int64_t* h_offsets, int32_t* h_counts, void* stream) {
  fdas_status st = check_trials(p, h_trials, count, false);
  if (st != FDAS_OK) return st;
  if (!h_offsets) return fail(FDAS_ERR_INVALID_ARG, "h_offsets is NULL");
  if (h_capacity < 0 || (h_capacity > 0 && !h_out)) return fail(FDAS_ERR_INVALID_ARG, "bad host output buffer");
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nh = p->desc.n_harm;
  const int cap = p->desc.cand_capacity;
  hipError_t e = ensure_streams(p);
  if (e != hipSuccess) return hip_fail(e, "creating the batch streams");
  // gather every trial's counts on the device, then one copy
  if (p->stage_done && p->h_stage) (void)hipEventSynchronize(p->stage_done);
  e = ensure_tables(p, 1, (size_t)count * sizeof(int32_t*));
  if (e != hipSuccess) return hip_fail(e, "allocating the batch staging area");
  if (count > p->counts_cap) {
    if (p->d_cand_ptrs) (void)hipFree(p->d_cand_ptrs);
    if (p->d_counts_all) (void)hipFree(p->d_counts_all);
    if (p->h_counts_all) (void)hipHostFree(p->h_counts_all);
    p->d_cand_ptrs = nullptr;
    p->d_counts_all = nullptr;
    p->h_counts_all = nullptr;
    p->counts_cap = 0;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_cand_ptrs), count * sizeof(int32_t*))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&p->d_counts_all), (size_t)count * 8 * sizeof(int32_t))) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&p->h_counts_all), (size_t)count * 8 * sizeof(int32_t), 0)) !=
            hipSuccess)
      return hip_fail(e, "allocating the batch count buffers");
    p->counts_cap = count;
  }
  int32_t** stage = static_cast<int32_t**>(p->h_stage);
  for (int i = 0; i < count; ++i) stage[i] = h_trials[i].d_counts;
  if ((e = hipMemcpyAsync(p->d_cand_ptrs, stage, count * sizeof(int32_t*), hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipEventRecord(p->stage_done, s)) != hipSuccess ||
      (e = launch_gather_counts(reinterpret_cast<int32_t* const*>(p->d_cand_ptrs), count, nh, p->d_counts_all, s)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(p->h_counts_all, p->d_counts_all, (size_t)count * nh * sizeof(int32_t),
                          hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_fail(e, "reading the batch candidate counts");
  if (h_counts) std::memcpy(h_counts, p->h_counts_all, (size_t)count * nh * sizeof(int32_t));
  bool overflow = false;
  // record i of trial t lands at pre[t] + i of one trial-major array
  std::vector<int64_t> pre(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    int64_t tot = 0;
    for (int k = 0; k < nh; ++k) {
      const int c = p->h_counts_all[i * nh + k];
      if (c < 0) return fail(FDAS_ERR_DEVICE, "negative candidate count");
      if (c > cap) overflow = true;
      tot += std::min(c, cap);
    }
    pre[i + 1] = pre[i] + tot;
  }
  const int64_t M = pre[count];
  if (M > INT32_MAX / 2) return fail(FDAS_ERR_CAPACITY, "%lld candidates in one batch readback", (long long)M);
  if (sort_passes_batch(count, p->rows, p->bits_r) > 8)
    return fail(FDAS_ERR_INVALID_ARG, "batch sort key of %d trials does not fit 64 bits", count);
  fdas_cand* sorted = nullptr;
  if (M > 0) {
    // buffers: the per-trial table and sort space for M records (grown on demand)
    if (count > p->rb_tab_cap) {
      if (p->d_rb_tab) (void)hipFree(p->d_rb_tab);
      p->d_rb_tab = nullptr;
      p->rb_tab_cap = 0;
      if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_rb_tab), (size_t)count * sizeof(RbTrial))) != hipSuccess)
        return hip_fail(e, "allocating the readback table");
      p->rb_tab_cap = count;
    }
    if (M > p->rb_sort_cap) {
      if (p->d_bsort_a) (void)hipFree(p->d_bsort_a);
      if (p->d_bsort_b) (void)hipFree(p->d_bsort_b);
      if (p->d_bsort_hist) (void)hipFree(p->d_bsort_hist);
      if (p->d_bsort_totals) (void)hipFree(p->d_bsort_totals);
      p->d_bsort_a = p->d_bsort_b = nullptr;
      p->d_bsort_hist = p->d_bsort_totals = nullptr;
      p->rb_sort_cap = 0;
      const int64_t want = std::max<int64_t>(M + M / 4, 1 << 16);
      if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_bsort_a), (size_t)want * sizeof(fdas_cand))) != hipSuccess ||
          (e = hipMalloc(reinterpret_cast<void**>(&p->d_bsort_b), (size_t)want * sizeof(fdas_cand))) != hipSuccess ||
          (e = hipMalloc(reinterpret_cast<void**>(&p->d_bsort_hist),
                         (size_t)256 * sort_tile_count((int)want) * sizeof(int))) != hipSuccess ||
          (e = hipMalloc(reinterpret_cast<void**>(&p->d_bsort_totals), (size_t)256 * 8 * sizeof(int))) != hipSuccess)
        return hip_fail(e, "allocating the batch sort buffers");
      p->rb_sort_cap = want;
    }
    e = ensure_tables(p, 1, (size_t)count * sizeof(RbTrial));
    if (e != hipSuccess) return hip_fail(e, "allocating the batch staging area");
    RbTrial* tab = static_cast<RbTrial*>(p->h_stage);
    for (int i = 0; i < count; ++i)
      tab[i] = RbTrial{reinterpret_cast<const int4*>(h_trials[i].d_cands), h_trials[i].d_counts, pre[i], 0};
    if ((e = hipMemcpyAsync(p->d_rb_tab, tab, (size_t)count * sizeof(RbTrial), hipMemcpyHostToDevice, s)) !=
            hipSuccess ||
        (e = hipEventRecord(p->stage_done, s)) != hipSuccess)
      return hip_fail(e, "uploading the readback table");
    e = launch_sort_batch(p->d_rb_tab, count, cap, nh, (int)M, p->rows, p->desc.z_max, p->bits_r, p->d_bsort_a,
                          p->d_bsort_b, p->d_bsort_hist, p->d_bsort_totals, &sorted, s);
    if (e != hipSuccess) return hip_fail(e, "ordering candidates");
  }
  if (p->desc.top_k <= 0) {
    // one copy of the trial-major array; a short host buffer truncates the last trials
    const int64_t nw = std::min<int64_t>(M, h_capacity);
    for (int i = 0; i <= count; ++i) h_offsets[i] = std::min<int64_t>(pre[i], h_capacity);
    if (nw < M) overflow = true;
    if (nw > 0 && (e = hipMemcpyAsync(h_out, sorted, (size_t)nw * sizeof(fdas_cand), hipMemcpyDeviceToHost, s)) !=
                      hipSuccess)
      return hip_fail(e, "reading candidates");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading candidates");
  } else {
    std::vector<fdas_cand> all((size_t)M), keep;
    if (M > 0 && (e = hipMemcpyAsync(all.data(), sorted, (size_t)M * sizeof(fdas_cand), hipMemcpyDeviceToHost, s)) !=
                     hipSuccess)
      return hip_fail(e, "reading candidates");
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "reading candidates");
    int64_t pos = 0;
    for (int i = 0; i < count; ++i) {
      h_offsets[i] = pos;
      if (pre[i + 1] == pre[i]) continue;
      int off[9] = {0};
      for (int k = 0; k < nh; ++k) off[k + 1] = off[k] + std::min(p->h_counts_all[i * nh + k], cap);
      keep.clear();
      keep_top_k(all.data() + pre[i], off, nh, p->desc.top_k, keep);
      const int64_t nw = std::min<int64_t>((int64_t)keep.size(), h_capacity - pos);
      if (nw > 0) std::memcpy(h_out + pos, keep.data(), (size_t)nw * sizeof(fdas_cand));
      if (nw < (int64_t)keep.size()) overflow = true;
      pos += std::max<int64_t>(nw, 0);
    }
    h_offsets[count] = pos;
  }
  if (overflow) return fail(FDAS_ERR_CAPACITY, "a candidate list overflowed (device capacity or h_capacity)");
  return ok();
}

fdas_status fdas_set_tuning(fdas_plan* p, const fdas_tuning* t) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  fdas_tuning v{};
  if (t) {
    v = *t;
    if (v.conv_templates_per_item < 0 || v.conv_templates_per_item > p->rows)
      return fail(FDAS_ERR_INVALID_ARG, "conv_templates_per_item %d outside [0, %d]", v.conv_templates_per_item, p->rows);
    if (v.conv_waves_per_simd < 0 || v.conv_waves_per_simd > 2)
      return fail(FDAS_ERR_INVALID_ARG, "conv_waves_per_simd %d outside [0, 2]", v.conv_waves_per_simd);
    if (v.ols_chunk != 0 && !ols_chunk_built(v.ols_chunk))
      return fail(FDAS_ERR_UNSUPPORTED, "ols_chunk %d: the built chunk lengths are 2048, 4096 and 8192", v.ols_chunk);
    if (v.ols_chunk != 0 && v.ols_chunk - (p->L_max - 1) < 1024)
      return fail(FDAS_ERR_INVALID_ARG, "ols_chunk %d leaves fewer than 1024 valid outputs", v.ols_chunk);
    if (v.hsum_tile != 0 && !harmsum_tile_built(v.hsum_tile))
      return fail(FDAS_ERR_UNSUPPORTED, "hsum_tile %d: the built tile widths are 256, 512 and 1024", v.hsum_tile);
    if (v.overlap_groups < 0 || v.overlap_groups > kMaxGroups)
      return fail(FDAS_ERR_INVALID_ARG, "overlap_groups %d outside [0, %d]", v.overlap_groups, kMaxGroups);
    if (v.emit_workgroups != 0 && (v.emit_workgroups < 64 || v.emit_workgroups > 16384))
      return fail(FDAS_ERR_INVALID_ARG, "emit_workgroups %d outside [64, 16384]", v.emit_workgroups);
  }
  p->tuning = v;
  return ok();
}

fdas_status fdas_autotune(fdas_plan* p, const fdas_trial* h_trials, int32_t count, int32_t repeats, fdas_tuning* out,
                          void* stream) {
  fdas_status st = check_trials(p, h_trials, count, true);
  if (st != FDAS_OK) return st;
  if (repeats < 1) return fail(FDAS_ERR_INVALID_ARG, "repeats must be >= 1");
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return hip_fail(e, "creating timing events");
  }
  const fdas_tuning saved = p->tuning;
  auto time_it = [&](const fdas_tuning& cand, double* ms) -> fdas_status {
    p->tuning = cand;
    fdas_status r = search_batch(p, h_trials, count, s);  // records the graph for this shape
    if (r != FDAS_OK) return r;
    hipError_t er = hipEventRecord(e0, s);
    for (int k = 0; k < repeats && r == FDAS_OK; ++k) r = search_batch(p, h_trials, count, s);
    if (r != FDAS_OK) return r;
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float t = 0.0f;
    if (er == hipSuccess) er = hipEventElapsedTime(&t, e0, e1);
    if (er != hipSuccess) return hip_fail(er, "timing a batch setting");
    *ms = t / repeats;
    return FDAS_OK;
  };
  fdas_tuning best{};
  double best_ms = 1e300;
  auto consider = [&](const fdas_tuning& cand) -> fdas_status {
    double ms = 0.0;
    fdas_status r = time_it(cand, &ms);
    if (r == FDAS_OK && ms < best_ms) {
      best_ms = ms;
      best = cand;
    }
    return r;
  };
  // 1. chunk length x waves per SIMD (one forward FFT per chunk a workgroup's
  //    range touches, no overlap); the chunk lengths whose overlap leaves
  //    fewer than 1024 valid outputs are skipped
  for (int C : {2048, 4096, 8192}) {
    if (C - (p->L_max - 1) < 1024) continue;
    for (int wps : {1, 2}) {
      fdas_tuning c{};
      c.ols_chunk = C;
      c.conv_waves_per_simd = wps;
      c.overlap_groups = 1;
      if ((st = consider(c)) != FDAS_OK) break;
    }
    if (st != FDAS_OK) break;
  }
  // 2. templates per forward FFT, 3. harmonic-sum tile width
  if (st == FDAS_OK) {
    const fdas_tuning base = best;
    for (int tpg : {5, 9, 17, 29, 43}) {
      if (tpg > p->rows) continue;
      fdas_tuning c = base;
      c.conv_templates_per_item = tpg;
      if ((st = consider(c)) != FDAS_OK) break;
    }
  }
  if (st == FDAS_OK && graphable(p)) {
    const fdas_tuning base = best;
    for (int cols : {256, 512}) {
      fdas_tuning c = base;
      c.hsum_tile = cols;
      if ((st = consider(c)) != FDAS_OK) break;
    }
  }
  // 4. overlap groups, 5. emission workgroups
  if (st == FDAS_OK && graphable(p)) {
    const fdas_tuning base = best;
    for (int g : {2, 4, 8}) {
      if (g > count) break;
      fdas_tuning c = base;
      c.overlap_groups = g;
      if ((st = consider(c)) != FDAS_OK) break;
    }
    const fdas_tuning base2 = best;
    for (int eb : {256, 4096}) {
      if (st != FDAS_OK) break;
      fdas_tuning c = base2;
      c.emit_workgroups = eb;
      st = consider(c);
    }
  }
  if (st == FDAS_OK) {
    // report the values the defaults stand for
    if (best.ols_chunk == 0) best.ols_chunk = p->ols[p->ols_idx].geom.C;
    if (best.conv_waves_per_simd == 0) best.conv_waves_per_simd = 2;
    if (best.hsum_tile == 0) best.hsum_tile = 1024;
    if (best.overlap_groups == 0) best.overlap_groups = 1;
    if (best.emit_workgroups == 0) best.emit_workgroups = 1024;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != FDAS_OK) {
    p->tuning = saved;
    return st;
  }
  p->tuning = best;
  if (out) *out = best;
  return ok();
}

}  // extern "C"
