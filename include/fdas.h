/*
 * fdas.h -- C ABI of libfdas, the MI355X (gfx950) FDAS hot path.
 *
 * FDAS (Fourier-domain acceleration search) as described by Wang, Thiagaraj &
 * Sinnen, "Combining Multiple Optimized FPGA-based Pulsar Search Modules Using
 * OpenCL", has two steps, and this library exposes one call for each:
 *
 *   fdas_convolve      Section 2.1 (eq. (1) / eq. (2)): the complex spectrum is
 *                      correlated with N_temp = 2*z_max+1 acceleration templates
 *                      (85 in Table 1) and the power of every output is written
 *                      to the filter-output plane (FOP), rows = templates,
 *                      columns = Fourier bins.
 *   fdas_harmonic_sum  Section 2.2, Algorithm 1: the FOP is stretched by
 *                      k = 1..N_hp (8 in Table 1), the harmonic planes
 *                      HP_k = HP_{k-1} + SP_k are formed without being stored,
 *                      every cell is compared with the threshold TA(k, i), and
 *                      cells above it are appended to per-plane candidate lists.
 *   fdas_candidates    copies the lists back and returns them in the loop order
 *                      of Algorithm 1, (k, i, j), optionally keeping N_cand per
 *                      plane (200 in Table 1).
 *
 * Conventions (all calls):
 *   - Every pointer named d_* is device memory on the plan's device, allocated
 *     and owned by the caller.  h_* pointers are host memory owned by the caller.
 *     The plan owns its templates, twiddle tables and workspace.
 *   - Arguments are validated before anything is launched; on error nothing
 *     has been written and the call has no side effect.  fdas_last_error()
 *     returns a thread-local message describing the last failure.
 *   - fdas_convolve and fdas_harmonic_sum are asynchronous on `stream`
 *     (a hipStream_t; NULL = the default stream).  fdas_plan_create,
 *     fdas_plan_destroy and fdas_candidates synchronise.
 *   - A plan may be used from one stream at a time (not re-entrant).
 *   - Readings of passages the paper leaves open (template formula, z step,
 *     alignment, stretch, thresholds) are fixed by this library as stated at
 *     each call.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDAS_ABI_VERSION 2

typedef enum {
  FDAS_OK = 0,
  FDAS_ERR_INVALID_ARG = 1,   /* bad pointer, size, layout or descriptor field */
  FDAS_ERR_NO_DEVICE = 2,     /* no usable GPU, or desc.device out of range */
  FDAS_ERR_OUT_OF_MEMORY = 3, /* device or host allocation failed */
  FDAS_ERR_DEVICE = 4,        /* a HIP runtime call failed */
  FDAS_ERR_CAPACITY = 5,      /* a candidate list overflowed (counts stay exact) */
  FDAS_ERR_UNSUPPORTED = 6    /* valid request that this build does not provide */
} fdas_status;

/* FT-convolution method (Section 2.1). */
typedef enum {
  FDAS_CONV_AUTO = 0,        /* the faster of the two on this GPU (overlap-save) */
  FDAS_CONV_OLS_FFT = 1,     /* overlap-save FFT correlation (Section 2.1.2, eq. (2)) */
  FDAS_CONV_DIRECT_MFMA = 2  /* direct complex FIR sum on the matrix cores (eq. (1)) */
} fdas_conv_method;

/* Arithmetic of the direct method (the overlap-save method is always FP32).
 * The split forms carry every operand value v as hi = round16(v) and
 * lo = round16(v - hi) and each product as hi*hi + hi*lo + lo*hi on the 16-bit
 * matrix cores with FP32 accumulation (FP16 operands are scaled by exact
 * powers of two per workgroup strip and per template tile). */
typedef enum {
  FDAS_PREC_FP32 = 0,
  FDAS_PREC_SPLIT_FP16 = 1,
  FDAS_PREC_SPLIT_BF16 = 2
} fdas_precision;

/* Harmonic index map used by fdas_harmonic_sum.  Algorithm 1 names a
 * stretch() it does not define; STRETCH is the literal reading used by
 * default, the other two follow the physics of a signal whose m-th harmonic
 * sits at (m z, m r). */
typedef enum {
  FDAS_HSUM_STRETCH = 0,     /* HP_k = HP_{k-1} + FOP(trunc(i/k), floor(j/k)) */
  FDAS_HSUM_FUNDAMENTAL = 1, /* HP_k = HP_{k-1} + FOP(k i, k j), 0 outside the plane */
  FDAS_HSUM_HIGHEST = 2      /* HP_k = sum_{m<=k} FOP(rho(m i, k), rho(m j, k)), rho = nearest,
                                halves away from zero; not cumulative */
} fdas_hsum_index;

typedef struct {
  int32_t struct_size;   /* sizeof(fdas_plan_desc); guards ABI drift */
  int64_t n_max;         /* largest spectrum length the plan accepts; 1 .. 2^30, and
                            (2*z_max+1) * n_max < 2^31 so that per-plane counts stay exact */
  int32_t z_max;         /* templates z = -z_max..z_max (row = z + z_max); 0..64, default 42 */
  int32_t n_harm;        /* harmonic planes N_hp, 1..8, default 8 */
  double  p_fa;          /* per-cell false-alarm probability of the default TA, (0, 1) */
  int32_t cand_capacity; /* candidates stored per plane on the device, 1 .. 2^22 */
  int32_t top_k;         /* readback keeps this many per plane (0 = all; 200 = Table 1) */
  fdas_conv_method method;
  fdas_precision precision;
  fdas_hsum_index hsum_index;
  int32_t ols_chunk;     /* overlap-save FFT length C: 2048, 4096 or 8192 (0 = 4096); C - (L_max - 1) >= 1024 */
  int32_t device;        /* HIP device ordinal */
} fdas_plan_desc;

/* One candidate: harmonic plane k (1-based), template z (= row - z_max),
 * Fourier bin r, and the FP32 harmonic sum HP_k(z, r).  16 bytes. */
typedef struct {
  int32_t harm;
  int32_t z;
  int32_t r;
  float power;
} fdas_cand;

typedef struct fdas_plan fdas_plan;

/* Fill *desc with the defaults: z_max 42, n_harm 8, p_fa 1e-6, n_max 2^22,
 * cand_capacity 65536, top_k 0, AUTO method, FP32, stretch index, device 0. */
void fdas_plan_desc_default(fdas_plan_desc* desc);

/* Create a plan (Table 1 sizes by default).  Builds the 2*z_max+1 templates in
 * FP64 from the Fourier-domain acceleration response (the paper names the
 * Ransom et al. correlation technique without printing coefficients):
 *   A(q, z) = integral_0^1 exp(i*pi*(z u^2 + (2q - z) u)) du,
 *   h_z[d]  = conj(A(-d, z)) / sqrt(sum_d |A(-d, z)|^2),
 *   d in [-L/2, L/2 - 1],  L(z) = 2*(8 + ceil(4.5*|z|))  (<= 400 taps, Section 1),
 * their overlap-save spectra, the default thresholds TA(k, i) = Q^{-1}(k, p_fa)
 * (inverse regularised upper incomplete gamma), and uploads them.
 * Returns FDAS_ERR_NO_DEVICE when no GPU is present; *out is NULL on error. */
fdas_status fdas_plan_create(const fdas_plan_desc* desc, fdas_plan** out);

/* Release a plan and its device memory.  NULL is a no-op.  Synchronises. */
fdas_status fdas_plan_destroy(fdas_plan* plan);

/* FT convolution + power (Section 2.1, eq. (1)/(2); power as in Section 2.2):
 *   d_fop[(z + z_max) * ld + j] = | sum_d X[j + d] h_z[d] |^2,  j in [0, n),
 * X[k] = 0 outside [0, n) (both ends zero-extended), column j = bin j.
 * d_spectrum: complex64[n] (interleaved re, im), 8-byte aligned.
 * d_fop: float[(2*z_max+1) * ld], 16-byte aligned, ld >= n and ld % 4 == 0.
 * 1 <= n <= n_max.  Asynchronous on stream.  Columns >= n are not written. */
fdas_status fdas_convolve(fdas_plan* plan, const void* d_spectrum, int64_t n,
                          float* d_fop, int64_t ld, void* stream);

/* Harmonic summing with threshold detection (Algorithm 1, Section 2.2):
 *   HP_1 = FOP, HP_k(i, j) = HP_{k-1}(i, j) + FOP(trunc(i/k), floor(j/k)),
 * summed in FP32 in k order (the plan's hsum_index selects another index map,
 * see FDAS_HSUM_*; sums are then in m order); a cell with HP_k(i, j) > TA(k, i)
 * is appended to list k-1.  d_ta: float[n_harm][2*z_max+1] or NULL for the plan's default.
 * d_cands: fdas_cand[n_harm][cand_capacity]; d_counts: int32[n_harm].
 * d_counts is reset by this call and ends holding the true number of cells
 * above threshold per plane, also when that exceeds cand_capacity (then only
 * cand_capacity records, in no particular order, are stored).  The order of
 * records inside a list is unspecified; fdas_candidates sorts them.
 * Same FOP layout rules as fdas_convolve.  Asynchronous on stream. */
fdas_status fdas_harmonic_sum(fdas_plan* plan, const float* d_fop, int64_t n, int64_t ld,
                              const float* d_ta, fdas_cand* d_cands, int32_t* d_counts,
                              void* stream);

/* fdas_harmonic_sum for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops and harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as fdas_harmonic_sum; it
 * calls no allocating routine.  Its scratch (hit-row counter, tile order and
 * hit-row list, 16.02 MiB) is a static device array of the library, one per
 * GPU, held until the process ends; calls that overlap on one GPU share it
 * and race, so they must be ordered (one stream, or events).  The array keeps
 * the last call's contents; every call clears the counter and rewrites the
 * tile order with kernels (no memset).  n <= 2^22 (FDAS_ERR_INVALID_ARG
 * otherwise).  Asynchronous on stream. */
fdas_status fdas_harmonic_sum_noalloc(fdas_plan* plan, const float* d_fop, int64_t n, int64_t ld,
                                      const float* d_ta, fdas_cand* d_cands, int32_t* d_counts,
                                      void* stream);

/* Copy the candidate lists back (after the work queued on stream), order them
 * by (harm, z, r) and write at most h_capacity records to h_out.  With
 * top_k > 0 each plane keeps its top_k highest powers (ties: lower z, then
 * lower r, first; N_cand of Table 1), selected on the device, still in
 * (harm, z, r) order.  *h_n receives the number written.
 * h_counts (optional, int32[n_harm]; NULL to skip) receives the device counts,
 * the true per-plane totals that tell a caller how much an overflowed list
 * lost; they are read in the same wait as the records.
 * Returns FDAS_ERR_CAPACITY if a device list overflowed or h_capacity was too
 * small; the records returned are then still ordered but incomplete. */
fdas_status fdas_candidates(fdas_plan* plan, const fdas_cand* d_cands, const int32_t* d_counts,
                            fdas_cand* h_out, int64_t h_capacity, int64_t* h_n,
                            int32_t* h_counts, void* stream);

/* --- batches of dispersion trials ------------------------------------------
 * A beam yields one spectrum per dispersion-measure trial (Table 1),
 * searched independently.  The batch calls run the same two steps as
 * fdas_convolve + fdas_harmonic_sum (identical arithmetic, so identical
 * results) for many spectra of uneven length at once: one persistent
 * convolution launch works through a queue of (trial, chunk, template group)
 * items, one harmonic-sum launch covers every trial's column tiles, and the
 * sequence is replayed from a HIP graph.  Trials can be split into groups
 * whose harmonic sums overlap the next group's convolution (the pipeline
 * computing of Section 3.3, with one FOP buffer per trial). */

/* One trial of a batch.  All pointers are caller-owned device memory; the FOP,
 * candidate and count buffers of different trials of one call must not
 * overlap.  Layout rules as for fdas_convolve / fdas_harmonic_sum. */
typedef struct {
  const void* d_spectrum; /* complex64[n] */
  int64_t n;              /* 1 <= n <= n_max */
  float* d_fop;           /* [2*z_max+1][ld] */
  int64_t ld;             /* >= n, multiple of 4 */
  fdas_cand* d_cands;     /* [n_harm][cand_capacity] */
  int32_t* d_counts;      /* [n_harm], reset by the call */
} fdas_trial;

/* Launch parameters chosen by fdas_autotune (all fields 0 = built-in default). */
typedef struct {
  int32_t conv_templates_per_item; /* at most this many templates share one forward FFT (1..2*z_max+1; 0 = all of a chunk's templates in a workgroup's range) */
  int32_t conv_waves_per_simd;     /* resident convolution waves per SIMD (1..2; default 2) */
  int32_t overlap_groups;          /* trial groups whose harmonic sums overlap later convolutions (1..8) */
  int32_t emit_workgroups;         /* workgroups of the candidate-emission pass (64..16384) */
  int32_t ols_chunk;               /* overlap-save chunk length C of the batch (2048, 4096, 8192; 0 = the plan's) */
  int32_t hsum_tile;               /* columns per harmonic-sum workgroup tile (256, 512, 1024; 0 = 1024) */
} fdas_tuning;

/* Convolution + harmonic sum (default thresholds) of `count` trials,
 * asynchronous on `stream`.  1 <= count <= 1024.  Equivalent to calling
 * fdas_convolve and fdas_harmonic_sum for each trial in turn.  The first call
 * with a new batch shape records a HIP graph (this call then synchronises);
 * later calls with the same shape replay it. */
fdas_status fdas_search_batch(fdas_plan* plan, const fdas_trial* h_trials, int32_t count, void* stream);

/* Ordered candidates of every trial of a batch in one readback: records of
 * trial t occupy h_out[h_offsets[t] .. h_offsets[t+1]) in (harm, z, r) order.
 * h_offsets: int64[count + 1]; h_counts (optional): int32[count][n_harm], the
 * device counts.  top_k applies per trial and plane.  Synchronises.  Returns
 * FDAS_ERR_CAPACITY if a device list overflowed or h_capacity was too small
 * (the records returned are then ordered but incomplete). */
fdas_status fdas_candidates_batch(fdas_plan* plan, const fdas_trial* h_trials, int32_t count, fdas_cand* h_out,
                                  int64_t h_capacity, int64_t* h_offsets, int32_t* h_counts, void* stream);

/* Time the batch path on these trials (their buffers are overwritten) over a
 * set of launch parameters -- the overlap-save chunk length C (the N_OLS-FT
 * of Section 2.1.2), the convolution's waves per SIMD and templates per
 * forward FFT, the harmonic-sum tile width, the overlap groups (Section 3.3)
 * and the emission grid -- keep the fastest in the plan for later batch
 * calls, and report it in *out (optional).  `repeats` timed runs per
 * setting (>= 1).  Results do not depend on the setting (every chunk length
 * computes the same correlation within FP32 rounding; candidates differ only
 * where a sum lies within rounding of its threshold).  Synchronises. */
fdas_status fdas_autotune(fdas_plan* plan, const fdas_trial* h_trials, int32_t count, int32_t repeats,
                          fdas_tuning* out, void* stream);

/* Set the launch parameters of the batch path by hand (NULL = defaults). */
fdas_status fdas_set_tuning(fdas_plan* plan, const fdas_tuning* tuning);

/* As fdas_candidates, but the ordered records land in a page-locked buffer
 * owned by the plan, written by the device itself, so the call waits once
 * (no intermediate wait for the counts).  *h_view points at *h_n records in
 * (harm, z, r) order, valid until the plan's next fdas_candidates_mapped or
 * fdas_plan_destroy.  h_counts as in fdas_candidates.  With top_k > 0 each
 * plane keeps its top_k highest powers as in fdas_candidates.  Synchronises. */
fdas_status fdas_candidates_mapped(fdas_plan* plan, const fdas_cand* d_cands, const int32_t* d_counts,
                                   const fdas_cand** h_view, int64_t* h_n, int32_t* h_counts, void* stream);

/* --- learned block pre-screen -----------------------------------------------
 * Not part of the paper's method: a small 1D convolutional network over the
 * zero-drift power of 4096-bin blocks that predicts whether the full search
 * would find a significant candidate in a block, so that the full search can
 * run on flagged blocks only (fdas_search_blocks).
 *   input a0[t] = log(1 + |X[4096 b + t]|^2)  (the template z = 0 is a unit delta,
 *                 so this is the FOP row z = 0)
 *   a_l = maxpool4(relu(conv(a_{l-1}))), l = 1..3 (1 -> 32 -> 32 -> 32 channels,
 *   kernel 9, zero padding 4); h = max_t relu(conv(a_3)); logit = wf.h + bf.
 *   Loss: weighted logistic, pos_weight * y * softplus(-l) + (1 - y) * softplus(l),
 *   mean over the batch.  Parameters: FP32 master copy, BF16 copy used by every
 *   kernel (FP32 accumulation), Adam updates.  Flat parameter order: W1[32][1][9],
 *   b1, W2[32][32][9], b2, W3, b3, W4, b4, wf[32], bf (fdas_prescreen_param_count). */
typedef struct fdas_prescreen fdas_prescreen;

int32_t fdas_prescreen_param_count(void);
/* Workspace for batches of up to max_batch blocks on `device`; parameters start at 0. */
fdas_status fdas_prescreen_create(int32_t device, int32_t max_batch, fdas_prescreen** out);
fdas_status fdas_prescreen_destroy(fdas_prescreen* ps);             /* NULL is a no-op */
/* FP32 parameters from / to host memory (set also clears the Adam state).  Synchronise. */
fdas_status fdas_prescreen_set_params(fdas_prescreen* ps, const float* h_theta);
fdas_status fdas_prescreen_get_params(fdas_prescreen* ps, float* h_theta);
/* d_features[i][t] = log(1 + |X[4096 h_blocks[i] + t]|^2) (0 past n), float[nblocks][4096].
 * h_blocks NULL: blocks 0 .. nblocks-1 (asynchronous); otherwise the list is
 * uploaded synchronously. */
fdas_status fdas_prescreen_features(fdas_prescreen* ps, const void* d_spectrum, int64_t n, const int32_t* h_blocks,
                                    int32_t nblocks, float* d_features, void* stream);
/* d_logits[i] for nblocks feature blocks (asynchronous). */
fdas_status fdas_prescreen_forward(fdas_prescreen* ps, const float* d_features, int32_t nblocks, float* d_logits,
                                   void* stream);
/* d_logits[b] for blocks b = 0 .. nblocks-1 of the spectrum (n complex FP32
 * bins on the device, 8-byte aligned), nblocks <= ceil(n / 4096):
 * fdas_prescreen_features followed by fdas_prescreen_forward in one kernel,
 * with no features buffer and no limit from max_batch; the same logits bit
 * for bit.  Asynchronous. */
fdas_status fdas_prescreen_infer(fdas_prescreen* ps, const void* d_spectrum, int64_t n, int32_t nblocks,
                                 float* d_logits, void* stream);
/* Logits, mean loss (d_loss[0]) and, if d_grad != NULL, the mean gradient (float[param_count]). */
fdas_status fdas_prescreen_gradient(fdas_prescreen* ps, const float* d_features, const float* d_labels,
                                    int32_t nblocks, float pos_weight, float* d_logits, float* d_loss, float* d_grad,
                                    void* stream);
/* One Adam step (beta 0.9 / 0.999) with learning rate lr on this batch. */
fdas_status fdas_prescreen_train_step(fdas_prescreen* ps, const float* d_features, const float* d_labels,
                                      int32_t nblocks, float pos_weight, float lr, float* d_logits, float* d_loss,
                                      void* stream);

/* The two-step search restricted to the listed 4096-bin blocks (h_blocks, any
 * order, duplicates allowed): the convolution runs on the overlap-save chunks
 * covering the listed blocks and the columns floor(j/k) their harmonic sums
 * read, the harmonic sum and compaction on the listed blocks' columns only, so
 * every candidate reported is one fdas_convolve + fdas_harmonic_sum would
 * report, with the same power.  FOP columns outside those chunks are not
 * written, and chunks that only hold the stretched sources of the listed
 * blocks are convolved for the rows the stretched map reads (z = -21..21 of
 * -42..42) only.  Plans other than overlap-save / 85 rows / stretch search
 * the whole spectrum.  Asynchronous (the block lists are uploaded
 * synchronously). */
fdas_status fdas_search_blocks(fdas_plan* plan, const void* d_spectrum, int64_t n, float* d_fop, int64_t ld,
                               const int32_t* h_blocks, int32_t nblocks, fdas_cand* d_cands, int32_t* d_counts,
                               void* stream);

/* The same restricted search with the block selection on the device, so
 * nothing waits for the host between the pre-screen and the search: blocks b
 * with d_logits[b] > threshold (d_logits: float[ceil(n/4096)] on the device,
 * e.g. written by fdas_prescreen_infer over blocks 0, 1, ...) and their
 * harmonic closure (as fdas_block_closure) are searched exactly as
 * fdas_search_blocks searches that block list (identical candidates and
 * powers).
 * Fallback to the plain search: when the screen is disabled (d_logits NULL),
 * when any logit is not finite (a diverged or broken model) or when the
 * threshold is NaN, every block is searched, which returns exactly what
 * fdas_convolve + fdas_harmonic_sum return.
 * n <= 16384 * 4096 bins.  The plan keeps device lists sized for the
 * spectrum.  Plans other than overlap-save / 85 rows / stretch search the
 * whole spectrum.  Asynchronous on stream. */
fdas_status fdas_search_flagged(fdas_plan* plan, const void* d_spectrum, int64_t n, float* d_fop, int64_t ld,
                                const float* d_logits, float threshold, fdas_cand* d_cands, int32_t* d_counts,
                                void* stream);

/* Harmonic closure of a block list under the stretched index map (host only):
 * the listed 4096-bin blocks plus, for every listed block b and m = 2..n_harm,
 * the blocks holding columns m*j .. m*j + m - 1 of its columns j (a signal at
 * column j raises the harmonic sums there), clipped to a spectrum of n bins.
 * h_out receives the distinct blocks in increasing order (*n_out of them;
 * at most ceil(n / 4096)).  Returns FDAS_ERR_CAPACITY, with *n_out the size
 * needed, if capacity is too small. */
fdas_status fdas_block_closure(int64_t n, int32_t n_harm, const int32_t* h_blocks, int32_t nblocks,
                               int32_t* h_out, int32_t capacity, int32_t* n_out);

/* Initial network parameters (host only): He-uniform convolution weights
 * (bound sqrt(6 / fan_in)), head weights uniform in +-1/sqrt(32), zero biases,
 * drawn from a splitmix64 stream seeded with `seed`, in the flat order of
 * fdas_prescreen_param_count.  h_theta: float[fdas_prescreen_param_count()]. */
fdas_status fdas_prescreen_init_params(uint64_t seed, float* h_theta);

/* Thread-local description of the last error of this thread ("" if none). */
const char* fdas_last_error(void);

/* --- host-only queries (no GPU needed) ------------------------------------ */

/* FDAS_ABI_VERSION of the loaded library. */
int32_t fdas_abi_version(void);

/* FP64 taps of template z (the coefficients fdas_plan_create uploads, before
 * rounding to FP32): taps[2*t] = Re h_z[d], taps[2*t+1] = Im h_z[d] for
 * d = -L/2 + t, t in [0, L).  capacity counts complex taps; *n_taps gets L.
 * |z| <= 64. */
fdas_status fdas_template_taps(int32_t z, double* taps, int32_t capacity, int32_t* n_taps);

/* Default thresholds T_k = Q^{-1}(k, p_fa), k = 1..n_harm, in FP64. */
fdas_status fdas_thresholds(int32_t n_harm, double p_fa, double* out);

#ifdef __cplusplus
}
#endif

#endif /* FDAS_H */
