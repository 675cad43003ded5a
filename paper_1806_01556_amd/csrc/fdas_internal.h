// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fdas.h"

namespace fdas {

// ---- FP64 plan arithmetic (fdas_math.cpp) ---------------------------------
int tap_count(int z);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void template_taps(int z, std::vector<std::complex<double>>& h);
void template_bank(int z_max, std::vector<std::vector<std::complex<double>>>& bank);
void ols_spectra(const std::vector<std::vector<std::complex<double>>>& bank, int C, int P,
                 std::vector<float>& out);
double erlang_threshold(int k, double p_fa);

// Packed template operand of the direct (matrix-core) correlation: templates
// ordered by |z| (0, -1, 1, -2, 2, ...) in tiles of 8; tile g covers taps
// [-P_g, P_g - 1] in P_g pairs of 64 lane-ordered floats (zero-padded to a
// multiple of 8 pairs).  tiles[g] = {P_g, first pair, members, padded pairs};
// rows[8 g + t] = FOP row of member t.
void direct_pack(const std::vector<std::vector<std::complex<double>>>& bank, int z_max, std::vector<float>& Bpk,
                 std::vector<int>& tiles, std::vector<int>& rows, int* P_max, int* P8_max);

// ---- overlap-save geometry -------------------------------------------------
constexpr int kOlsC = 4096;      // default FFT length of one chunk

struct OlsGeom {
  int C;   // chunk FFT length
  int P;   // left context = max L/2
  int V;   // valid outputs per chunk = C - (L_max - 1)
};

// Device tables of one chunk length: template spectra [rows][C] and twiddles
// (tw1 [16][C/16] = w_C^(k t); tw2 [17][TW2] = w_M^(k c), M = C/16, TW2 = M/16,
// and in row 16 w32^p for the 8192-point transform).
struct OlsTables {
  OlsGeom geom{};
  float2* H = nullptr;
  float2* tw1 = nullptr;
  float2* tw2 = nullptr;
};

bool ols_chunk_built(int C);  // 2048, 4096, 8192
int ols_threads(int C);       // threads of a convolution workgroup (C / 16)
int ols_slots_per_cu(int C);  // resident convolution workgroups per compute unit
void fft_twiddles(int C, std::vector<float>& tw1, std::vector<float>& tw2);

// ---- kernel launchers (k_*.hip) -------------------------------------------
// slots: workgroups of the persistent grid (all resident at once).
hipError_t launch_ols_conv(const float2* x, int64_t n, float* fop, int64_t ld, const OlsTables& t, int rows,
                           int slots, hipStream_t s);

// Only the listed overlap-save chunks (chunk_list[0 .. nlist), device array)
// and templates (FOP rows) z0 .. z0 + nr - 1; zrow is the row of the
// zero-drift template (written as |X|^2).  With d_nlist the kernel reads
// the list length from device memory and nlist is only its upper bound (the
// grid is sized for it).
hipError_t launch_ols_conv_list(const float2* x, int64_t n, float* fop, int64_t ld, const OlsTables& t, int z0,
                                int nr, int zrow, int slots, const int* chunk_list, int nlist, hipStream_t s,
                                const int* d_nlist = nullptr);

// FOP rows the stretched harmonic sums read as sources (k = 2 .. nh) of an
// 2*Z+1-row plane: [*lo, *hi]; empty (lo > hi) when nh < 2.
void stretch_source_rows(int Z, int nh, int* lo, int* hi);

// One spectrum of a batch for the convolution queue (device table entry).
struct ConvTrial {
  const float2* x;
  float* fop;
  int64_t n;
  int64_t ld;
  int64_t item0;  // first (chunk, template) pair of this trial: pairs before it = sum of chunks * rows
};

// (chunk, template) pairs [item_begin, item_end) of a batch, split into equal
// contiguous ranges over the resident workgroups; at most tmax templates share
// one forward FFT (0: a whole chunk's templates).
hipError_t launch_ols_conv_batch(const ConvTrial* trials, int ntrials, int64_t item_begin, int64_t item_end,
                                 const OlsTables& t, int rows, int tmax, int slots, hipStream_t s);

// Split 16-bit form of the packed operand: templates ordered and tiled as in
// direct_pack; tile g covers 2 P8 taps in P8/8 groups of 16, each group 64
// lanes x 8 hi values then 64 x 8 lo values (16-bit patterns, lane group
// kg = lane/16 holding taps 4kg..4kg+3 as (Re, Im) pairs).  Tile values are
// scaled by 2^eh (largest magnitude brought to about 2^14); tscale[g] = 2^-eh.
// tiles[4g + 1] counts 16-tap groups.  bf16 selects bfloat16, else FP16.
void direct_pack_split(const std::vector<std::vector<std::complex<double>>>& bank, int z_max, bool bf16,
                       std::vector<uint16_t>& Bsp, std::vector<float>& tscale, std::vector<int>& tiles,
                       std::vector<int>& rows, int* P_max, int* P8_max);

struct DirectTables {
  const float* Bpk;    // packed template operand
  const int4* tiles;   // per tile {P, first pair, members, padded pairs}
  const int* rows;     // [ntiles][8] FOP rows
  int ntiles;
  int P_max;    // largest P over the tiles
  int P8_max;   // largest padded pair count
  const uint4* Bsp = nullptr;     // split 16-bit operand (split precisions)
  const float* tscale = nullptr;  // per-tile 2^-eh (split precisions)
};
int direct_block_bins();
int direct_max_half_taps();
size_t direct_lds_bytes(int P_max, int P8_max);
hipError_t launch_direct_conv(const float2* x, int64_t n, float* fop, int64_t ld, const DirectTables& t,
                              hipStream_t s);
hipError_t launch_direct_conv_split(const float2* x, int64_t n, float* fop, int64_t ld, const DirectTables& t,
                                    bool bf16, hipStream_t s);

// Columns handled by one workgroup of the 85-row harmonic-sum kernel.
int harmsum_tile_columns();

// Order in which the 85-row harmonic-sum kernel visits its column tiles of
// `cols` columns: tile_of_block[b] is the tile of workgroup b (-1: none).
void harmsum_tile_order(int64_t n, std::vector<int>& tile_of_block, int cols);
// Tile widths (columns) the 85-row batch harmonic sum is built for: 256, 512, 1024.
bool harmsum_tile_built(int cols);

// Workspace of the two-phase 85-row harmonic sum.
struct HsWork {
  const int* tile_of_block;  // workgroup -> column tile (-1: none)
  int blocks;                // workgroups of phase 1
  int4* hitrows;             // {j0, row mask words}: ceil(n/4) entries at most
  int32_t* hitrow_count;     // entries appended by phase 1
  int emit_blocks;           // workgroups of phase 2 (0: default)
};

// One spectrum of a batch for the harmonic sum (device table entry).
struct HsTrial {
  const float* fop;
  int64_t ld;
  fdas_cand* cands;
  int32_t* counts;
  const int* tile_of_block;  // this length's tile order
  int n;
  int block0;                // first phase-1 workgroup of this trial
  int nblocks;               // phase-1 workgroups of this trial
  int pad;
};

hipError_t launch_zero_counts_batch(const HsTrial* trials, int ntrials, int nh, hipStream_t s);

// Two-phase 85-row stretch sum over phase-1 workgroups [blk_begin, blk_end)
// of a batch (default thresholds ta, capacity cap per plane), column tiles of
// tile_cols columns (each trial's tile order built for that width).
hipError_t launch_harmsum_batch85(const HsTrial* trials, int ntrials, int blk_begin, int blk_end, int n_harm,
                                  const float* ta, int cap, int4* hitrows, int32_t* hitrow_count, int eblocks,
                                  int tile_cols, hipStream_t s);

// index: FDAS_HSUM_* (the stretch map uses the two-phase kernels for 85 rows).
// counts[0 .. n_harm) are reset by the launch.
hipError_t launch_harmsum(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm,
                          const float* ta, fdas_cand* cands, int cap, int32_t* counts,
                          const HsWork& wk, int index, hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int count, int32_t value, hipStream_t s);

// Allocation-free harmonic sum: the same kernels with their scratch (hit-row
// counter, tile order, hit-row list) in the library's static device array.
// harmsum_noalloc_scratch returns that array's address on the current device.
int64_t harmsum_noalloc_max_n();
size_t harmsum_noalloc_scratch_bytes();
hipError_t harmsum_noalloc_scratch(void** ptr);
hipError_t launch_harmsum_noalloc(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm, const float* ta,
                                  fdas_cand* cands, int cap, int32_t* counts, void* scratch, int emit_blocks,
                                  int index, hipStream_t s);

int sort_tile_count(int m);
int sort_passes(int rows, int bits_r);

// Ordered records [0, min(total, out_cap)) and the nh counts copied into
// device-visible page-locked host memory by a kernel; with keep > 0 every
// plane holds at most keep records (the layout launch_topk writes).
hipError_t launch_copy_out(const fdas_cand* sorted, int cap, int nh, const int32_t* counts, int out_cap,
                           fdas_cand* out, int32_t* counts_out, hipStream_t s, int keep = 0);

// Table 1's N_cand per plane on the device: from the ordered array (planes
// packed, min(count, cap) records each) keep each plane's top_k highest
// powers (ties: lower z, then lower r), in (z, r) order, packed into out
// (plane k after sum_{k' < k} min(top_k, its records)).
hipError_t launch_topk(const fdas_cand* sorted, int cap, int nh, const int32_t* counts, int top_k, fdas_cand* out,
                       hipStream_t s);

// out[t * nh + k] = ptrs[t][k] for t < count, k < nh
hipError_t launch_gather_counts(int32_t* const* ptrs, int count, int nh, int32_t* out, hipStream_t s);

// Pack the per-plane lists (planes + k*cap, min(counts[k], cap) records each,
// counts read on the device) into `a` and order them by (harm, z, r).  `b` is
// scratch of the same size (nh * cap records), `hist` holds
// 256 * sort_tile_count(nh * cap) ints, `totals` 256 * sort_passes ints.
// *sorted receives a or b.  Nothing waits for the host.
hipError_t launch_sort_candidates(const fdas_cand* planes, int cap, int nh, const int32_t* counts, int rows,
                                  int z_max, int bits_r, fdas_cand* a, fdas_cand* b, int* hist, int* totals,
                                  fdas_cand** sorted, hipStream_t s);

// One trial of a batch readback: its per-plane lists and device counts, and
// the index of its first record in the packed array (host prefix of the
// clamped counts).
struct RbTrial {
  const int4* cands;
  const int32_t* counts;
  int64_t off;
  int64_t pad;
};

int sort_passes_batch(int count, int rows, int bits_r);

// Order the lists of `count` trials (m records in all) as one trial-major
// array in (trial, harm, z, r) order.  a, b hold m records, hist
// 256 * sort_tile_count(m) ints, totals 256 * sort_passes_batch ints.
hipError_t launch_sort_batch(const RbTrial* tab, int count, int cap, int nh, int m, int rows, int z_max, int bits_r,
                             fdas_cand* a, fdas_cand* b, int* hist, int* totals, fdas_cand** sorted, hipStream_t s);

// ---- learned block pre-screen (k_prescreen.hip) ----------------------------
struct PsBuffers {
  float* theta;          // FP32 master parameters
  float* grad;           // gradient accumulator (mean over the batch)
  float* m;              // Adam moments
  float* v;
  unsigned short* wbf;   // BF16 copy used by the kernels
  unsigned short* wflip; // [32][32][9] transposed, flipped kernel of one layer
  unsigned short* wpack; // layers 1..3 as matrix-core A operands (kPsPackShorts)
  float *a1, *a2, *a3, *r4;               // activations [B][32][1024 / 256 / 64 / 64]
  unsigned char *arg1, *arg2, *arg3;      // max-pool positions
  float *dz1, *dz2, *dz3, *dz4;           // pre-activation gradients [B][32][4096 / 1024 / 256 / 64]
};
int ps_param_count();
constexpr int kPsPackShorts = 3 * 2 * 9 * 64 * 8;
// features of listed 4096-bin blocks: log(1 + |X|^2)
hipError_t ps_features(const float2* x, int64_t n, const int* blocks, int nb, float* out, hipStream_t s);
// forward (logits); with labels also the loss (atomically added, mean) and the gradient into pb.grad
hipError_t ps_forward_backward(const PsBuffers& pb, const float* feats, int nb, const float* labels, float pos_weight,
                               float* logits, float* loss, hipStream_t s);
// logits of blocks 0..nb-1 of an n-bin spectrum, the features computed in the inference kernel
hipError_t ps_infer_spectrum(const PsBuffers& pb, const float2* x, int64_t n, int nb, float* logits, hipStream_t s);
hipError_t ps_adam(const PsBuffers& pb, float lr, float b1, float b2, float c1, float c2, float eps, hipStream_t s);
hipError_t ps_round(const PsBuffers& pb, hipStream_t s);
hipError_t ps_zero(float* p, int n, hipStream_t s);

// Device-side block selection of the pre-screened search (one workgroup):
// from the logits of blocks 0..nblk-1 and a threshold, writes into `lists` the
// searched-chunk list (cap_c entries), the tile list (cap_t entries, unused
// tail -1), the source-only chunk list (cap_c entries) and the three counts.
// nblk <= kMaxSelBlocks.
constexpr int kMaxSelBlocks = 16384;
hipError_t ps_search_lists(const float* logits, float thr, int64_t n, int nblk, int nh, int V, int tcols, int* lists,
                           int cap_c, int cap_t, hipStream_t s);

}  // namespace fdas
