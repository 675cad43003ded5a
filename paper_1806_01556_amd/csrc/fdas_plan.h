// The plan object behind the C ABI and the host helpers shared by the
// single-spectrum calls (fdas_host.cpp) and the batch calls (fdas_batch.cpp).
#pragma once

#include <map>
#include <string>
#include <vector>

#include "fdas_internal.h"

struct fdas_plan {
  fdas_plan_desc desc;
  int device = 0;
  int rows = 0;          // 2*z_max + 1
  int L_max = 0;         // taps of the longest template
  int cus = 256;         // compute units of the device
  fdas::OlsTables ols[3];  // overlap-save tables per chunk length 2048, 4096, 8192 (built on demand)
  int ols_idx = 1;         // chunk length of the single-spectrum calls (the descriptor's)
  bool direct = false;      // FDAS_CONV_DIRECT_MFMA: matrix-core correlation instead of overlap-save
  float* d_Bpk = nullptr;   // direct: packed template operand
  int4* d_dtiles = nullptr; // direct: per-tile {P, first pair, members, 0}
  int* d_drows = nullptr;   // direct: [tiles][8] FOP rows
  int dtiles = 0, dP_max = 0, dP8_max = 0;
  uint4* d_Bsp = nullptr;   // direct, split precisions: hi/lo 16-bit operand
  float* d_tscale = nullptr;  // direct, split precisions: per-tile 2^-eh
  float* d_ta = nullptr;    // [n_harm][rows] default thresholds
  std::vector<float> h_ta;
  fdas_cand* d_sort_a = nullptr;  // [n_harm * cand_capacity] packed candidates
  fdas_cand* d_sort_b = nullptr;  // radix-sort ping-pong buffer
  int* d_sort_hist = nullptr;     // [256 * tiles] digit histograms
  int* d_sort_totals = nullptr;   // [256 * passes] digit totals per pass
  int32_t* h_counts = nullptr;    // pinned host copy of the device counts
  fdas_cand* h_result = nullptr;  // page-locked result records of fdas_candidates_mapped
  int32_t* h_result_counts = nullptr;
  int bits_r = 1;                 // bits of the column index in the sort key
  std::map<std::pair<int64_t, int>, std::pair<int*, int>> tile_orders;  // (n, tile columns) -> (device order, workgroups)
  int4* d_hitrows = nullptr;      // [ceil(n_max/4)] rows with hits (harmonic sum phase 1)
  int32_t* d_hitrow_count = nullptr;
  fdas_tuning tuning{};           // batch launch parameters (0 = default)
  int* d_lists = nullptr;         // fdas_search_blocks: chunk list then tile list
  int64_t list_cap = 0;

  // ---- batch path (fdas_batch.cpp) ----
  int batch_cap = 0;                     // trials the tables below hold
  fdas::ConvTrial* d_conv_trials = nullptr;
  fdas::HsTrial* d_hs_trials = nullptr;
  void* h_stage = nullptr;               // pinned staging of both tables
  size_t h_stage_bytes = 0;
  hipEvent_t stage_done = nullptr;       // last upload from h_stage has been consumed
  int4* d_bhitrows = nullptr;            // hit-row list of a batch
  int64_t bhitrows_cap = 0;
  int32_t* d_bhitrow_count = nullptr;
  fdas_cand** d_cand_ptrs = nullptr;     // candidates_batch: per-trial count pointers (as int32_t*)
  int32_t* d_counts_all = nullptr;       // candidates_batch: gathered counts [cap][n_harm]
  int32_t* h_counts_all = nullptr;       // pinned copy
  int counts_cap = 0;
  fdas::RbTrial* d_rb_tab = nullptr;     // candidates_batch: per-trial readback table
  int rb_tab_cap = 0;
  fdas_cand* d_bsort_a = nullptr;        // candidates_batch: sort buffers of rb_sort_cap records
  fdas_cand* d_bsort_b = nullptr;
  int* d_bsort_hist = nullptr;           // [256 * tiles]
  int* d_bsort_totals = nullptr;         // [256 * 8]
  int64_t rb_sort_cap = 0;
  hipStream_t cap_stream = nullptr;      // stream the batch graph is recorded on
  hipStream_t side_stream = nullptr;     // harmonic sums overlapping later convolutions
  std::vector<hipEvent_t> fork_events;   // one per overlap group, plus the join
  hipGraphExec_t graph_exec = nullptr;
  hipEvent_t graph_done = nullptr;       // recorded after every graph launch
  std::vector<int64_t> graph_key;        // launch shape the graph was recorded for
};

namespace fdas {

fdas_status fail(fdas_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fdas_status ok();
fdas_status hip_fail(hipError_t e, const char* what);
fdas_status check_fop_args(const fdas_plan* p, const void* fop, int64_t n, int64_t ld);
// device tile order of the 85-row harmonic sum for length n (cached in the plan)
hipError_t tile_order_for(fdas_plan* p, int64_t n, const int** d_order, int* blocks, int cols = 1024);
// paper mode: planes [off[k], off[k+1]) of `sorted` reduced to their top_k
// powers, appended to keep in (harm, z, r) order
void keep_top_k(const fdas_cand* sorted, const int* off, int nh, int top_k, std::vector<fdas_cand>& keep);
// release the batch-path resources of a plan
void free_batch(fdas_plan* p);

// Index of a chunk length in fdas_plan::ols (-1: not built).
inline int ols_index(int C) { return C == 2048 ? 0 : (C == 4096 ? 1 : (C == 8192 ? 2 : -1)); }
// The overlap-save tables of chunk length C, built and uploaded on first use
// (the plan's device current).
hipError_t ols_tables(fdas_plan* p, int C, const OlsTables** out);
// Persistent-grid workgroups of the convolution at chunk length C.
inline int ols_slots(const fdas_plan* p, int C) { return p->cus * ols_slots_per_cu(C); }

// Make the plan's device current for the duration of a call.
struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    err = hipGetDevice(&prev);
    if (err == hipSuccess && prev != dev) {
      err = hipSetDevice(dev);
      changed = err == hipSuccess;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

}  // namespace fdas
