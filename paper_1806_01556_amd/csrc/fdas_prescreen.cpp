// Learned block pre-screen (C ABI) and the block-restricted search it feeds.
//
// fdas_prescreen_* own the network's parameters (FP32 master, BF16 copy),
// Adam state and activation workspace for up to max_batch blocks of 4096
// bins.  fdas_search_blocks runs the full two-step search only on a set of
// blocks: the convolution on the overlap-save chunks that cover those blocks
// and the blocks their stretched harmonic sums read (floor(j/k), k <= n_harm),
// the harmonic sum and candidate compaction on the listed blocks' columns.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <set>
#include <vector>

#include "fdas_plan.h"

struct fdas_prescreen {
  int device = 0;
  int max_batch = 0;
  int step = 0;  // Adam steps taken
  fdas::PsBuffers pb{};
  std::vector<void*> allocs;
  int* d_blocks = nullptr;  // block list for fdas_prescreen_features
  int blocks_cap = 0;
};

using namespace fdas;

namespace {

void free_ps(fdas_prescreen* ps) {
  if (!ps) return;
  for (void* p : ps->allocs) (void)hipFree(p);
  if (ps->d_blocks) (void)hipFree(ps->d_blocks);
  delete ps;
}

template <typename T>
hipError_t alloc(fdas_prescreen* ps, T** p, size_t count) {
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return e;
  ps->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return hipSuccess;
}

constexpr int kBlock = 4096;

fdas_status check_batch(const fdas_prescreen* ps, int nb) {
  if (!ps) return fail(FDAS_ERR_INVALID_ARG, "pre-screen is NULL");
  if (nb < 1 || nb > ps->max_batch)
    return fail(FDAS_ERR_INVALID_ARG, "batch of %d blocks outside [1, %d]", nb, ps->max_batch);
  return FDAS_OK;
}

}  // namespace

extern "C" {

int32_t fdas_prescreen_param_count(void) { return ps_param_count(); }

fdas_status fdas_prescreen_create(int32_t device, int32_t max_batch, fdas_prescreen** out) {
  if (!out) return fail(FDAS_ERR_INVALID_ARG, "out pointer is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > 65536) return fail(FDAS_ERR_INVALID_ARG, "max_batch %d outside [1, 65536]", max_batch);
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(FDAS_ERR_NO_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(FDAS_ERR_NO_DEVICE, "device %d outside [0, %d)", device, ndev);
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  fdas_prescreen* ps = new (std::nothrow) fdas_prescreen();
  if (!ps) return fail(FDAS_ERR_OUT_OF_MEMORY, "host allocation failed");
  ps->device = device;
  ps->max_batch = max_batch;
  const size_t B = (size_t)max_batch, C = 32;
  const int np = ps_param_count();
  PsBuffers& b = ps->pb;
  if ((e = alloc(ps, &b.theta, np)) != hipSuccess || (e = alloc(ps, &b.grad, np)) != hipSuccess ||
      (e = alloc(ps, &b.m, np)) != hipSuccess || (e = alloc(ps, &b.v, np)) != hipSuccess ||
      (e = alloc(ps, &b.wbf, np)) != hipSuccess || (e = alloc(ps, &b.wflip, C * C * 9)) != hipSuccess ||
      (e = alloc(ps, &b.wpack, kPsPackShorts)) != hipSuccess ||
      (e = alloc(ps, &b.a1, B * C * 1024)) != hipSuccess || (e = alloc(ps, &b.a2, B * C * 256)) != hipSuccess ||
      (e = alloc(ps, &b.a3, B * C * 64)) != hipSuccess || (e = alloc(ps, &b.r4, B * C * 64)) != hipSuccess ||
      (e = alloc(ps, &b.arg1, B * C * 1024)) != hipSuccess || (e = alloc(ps, &b.arg2, B * C * 256)) != hipSuccess ||
      (e = alloc(ps, &b.arg3, B * C * 64)) != hipSuccess || (e = alloc(ps, &b.dz1, B * C * 4096)) != hipSuccess ||
      (e = alloc(ps, &b.dz2, B * C * 1024)) != hipSuccess || (e = alloc(ps, &b.dz3, B * C * 256)) != hipSuccess ||
      (e = alloc(ps, &b.dz4, B * C * 64)) != hipSuccess) {
    free_ps(ps);
    return hip_fail(e, "allocating the pre-screen workspace");
  }
  std::vector<float> zero(np, 0.0f);
  if ((e = hipMemcpy(b.theta, zero.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b.grad, zero.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b.m, zero.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(b.v, zero.data(), np * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = ps_round(b, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
    free_ps(ps);
    return hip_fail(e, "initialising the pre-screen parameters");
  }
  *out = ps;
  return ok();
}

fdas_status fdas_prescreen_destroy(fdas_prescreen* ps) {
  if (!ps) return ok();
  DeviceGuard dg(ps->device);
  (void)hipDeviceSynchronize();
  free_ps(ps);
  return ok();
}

fdas_status fdas_prescreen_set_params(fdas_prescreen* ps, const float* h_theta) {
  if (!ps || !h_theta) return fail(FDAS_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard dg(ps->device);
  const int np = ps_param_count();
  hipError_t e = hipMemcpy(ps->pb.theta, h_theta, np * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = ps_zero(ps->pb.m, np, nullptr);
  if (e == hipSuccess) e = ps_zero(ps->pb.v, np, nullptr);
  if (e == hipSuccess) e = ps_zero(ps->pb.grad, np, nullptr);
  if (e == hipSuccess) e = ps_round(ps->pb, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "setting the pre-screen parameters");
  ps->step = 0;
  return ok();
}

fdas_status fdas_prescreen_get_params(fdas_prescreen* ps, float* h_theta) {
  if (!ps || !h_theta) return fail(FDAS_ERR_INVALID_ARG, "NULL argument");
  DeviceGuard dg(ps->device);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h_theta, ps->pb.theta, ps_param_count() * sizeof(float), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading the pre-screen parameters");
  return ok();
}

fdas_status fdas_prescreen_features(fdas_prescreen* ps, const void* d_spectrum, int64_t n, const int32_t* h_blocks,
                                    int32_t nblocks, float* d_features, void* stream) {
  fdas_status st = check_batch(ps, nblocks);
  if (st != FDAS_OK) return st;
  if (!d_spectrum || !d_features || n < 1) return fail(FDAS_ERR_INVALID_ARG, "bad feature arguments");
  const int64_t nblk = (n + kBlock - 1) / kBlock;
  if (!h_blocks) {
    // blocks 0 .. nblocks-1: no list to upload, nothing waits for the host
    if (nblocks > nblk) return fail(FDAS_ERR_INVALID_ARG, "%d blocks > the spectrum's %lld", nblocks, (long long)nblk);
    DeviceGuard dg0(ps->device);
    hipError_t e0 = ps_features(static_cast<const float2*>(d_spectrum), n, nullptr, nblocks, d_features,
                                static_cast<hipStream_t>(stream));
    if (e0 != hipSuccess) return hip_fail(e0, "computing pre-screen features");
    return ok();
  }
  for (int i = 0; i < nblocks; ++i)
    if (h_blocks[i] < 0 || h_blocks[i] >= nblk) return fail(FDAS_ERR_INVALID_ARG, "block %d outside the spectrum", h_blocks[i]);
  DeviceGuard dg(ps->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  if (nblocks > ps->blocks_cap) {
    if (ps->d_blocks) (void)hipFree(ps->d_blocks);
    ps->d_blocks = nullptr;
    ps->blocks_cap = 0;
    if ((e = hipMalloc(reinterpret_cast<void**>(&ps->d_blocks), nblocks * sizeof(int))) != hipSuccess)
      return hip_fail(e, "allocating the block list");
    ps->blocks_cap = nblocks;
  }
  // the list is small; a synchronous copy keeps the host array's lifetime simple
  if ((e = hipStreamSynchronize(s)) != hipSuccess ||
      (e = hipMemcpy(ps->d_blocks, h_blocks, nblocks * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = ps_features(static_cast<const float2*>(d_spectrum), n, ps->d_blocks, nblocks, d_features, s)) != hipSuccess)
    return hip_fail(e, "computing pre-screen features");
  return ok();
}

fdas_status fdas_prescreen_forward(fdas_prescreen* ps, const float* d_features, int32_t nblocks, float* d_logits,
                                   void* stream) {
  fdas_status st = check_batch(ps, nblocks);
  if (st != FDAS_OK) return st;
  if (!d_features || !d_logits) return fail(FDAS_ERR_INVALID_ARG, "NULL buffer");
  DeviceGuard dg(ps->device);
  hipError_t e = ps_forward_backward(ps->pb, d_features, nblocks, nullptr, 1.0f, d_logits, nullptr,
                                     static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "pre-screen forward");
  return ok();
}

fdas_status fdas_prescreen_infer(fdas_prescreen* ps, const void* d_spectrum, int64_t n, int32_t nblocks,
                                 float* d_logits, void* stream) {
  if (!ps) return fail(FDAS_ERR_INVALID_ARG, "pre-screen is NULL");
  if (!d_spectrum || reinterpret_cast<uintptr_t>(d_spectrum) % 8 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "spectrum pointer is NULL or not 8-byte aligned");
  if (!d_logits || reinterpret_cast<uintptr_t>(d_logits) % 4 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "logits pointer is NULL or misaligned");
  if (n < 1) return fail(FDAS_ERR_INVALID_ARG, "spectrum of %lld bins", (long long)n);
  const int64_t nblk = (n + kBlock - 1) / kBlock;
  if (nblocks < 1 || nblocks > nblk)
    return fail(FDAS_ERR_INVALID_ARG, "nblocks %d outside [1, %lld]", nblocks, (long long)nblk);
  DeviceGuard dg(ps->device);
  hipError_t e = ps_infer_spectrum(ps->pb, static_cast<const float2*>(d_spectrum), n, nblocks, d_logits,
                                   static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "pre-screen inference");
  return ok();
}

fdas_status fdas_prescreen_gradient(fdas_prescreen* ps, const float* d_features, const float* d_labels,
                                    int32_t nblocks, float pos_weight, float* d_logits, float* d_loss, float* d_grad,
                                    void* stream) {
  fdas_status st = check_batch(ps, nblocks);
  if (st != FDAS_OK) return st;
  if (!d_features || !d_labels || !d_logits || !d_loss) return fail(FDAS_ERR_INVALID_ARG, "NULL buffer");
  if (!(pos_weight > 0.0f)) return fail(FDAS_ERR_INVALID_ARG, "pos_weight must be > 0");
  DeviceGuard dg(ps->device);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int np = ps_param_count();
  hipError_t e = ps_zero(ps->pb.grad, np, s);
  if (e == hipSuccess) e = ps_zero(d_loss, 1, s);
  if (e == hipSuccess) e = ps_forward_backward(ps->pb, d_features, nblocks, d_labels, pos_weight, d_logits, d_loss, s);
  if (e == hipSuccess && d_grad)
    e = hipMemcpyAsync(d_grad, ps->pb.grad, np * sizeof(float), hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "pre-screen gradient");
  return ok();
}

fdas_status fdas_prescreen_train_step(fdas_prescreen* ps, const float* d_features, const float* d_labels,
                                      int32_t nblocks, float pos_weight, float lr, float* d_logits, float* d_loss,
                                      void* stream) {
  if (!(lr > 0.0f)) return fail(FDAS_ERR_INVALID_ARG, "lr must be > 0");
  fdas_status st = fdas_prescreen_gradient(ps, d_features, d_labels, nblocks, pos_weight, d_logits, d_loss, nullptr,
                                           stream);
  if (st != FDAS_OK) return st;
  ps->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)ps->step), c2 = 1.0f - std::pow(b2, (float)ps->step);
  hipError_t e = ps_adam(ps->pb, lr, b1, b2, c1, c2, 1e-8f, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "pre-screen update");
  return ok();
}

fdas_status fdas_block_closure(int64_t n, int32_t n_harm, const int32_t* h_blocks, int32_t nblocks, int32_t* h_out,
                               int32_t capacity, int32_t* n_out) {
  if (!n_out) return fail(FDAS_ERR_INVALID_ARG, "n_out is NULL");
  *n_out = 0;
  if (n < 1 || n > ((int64_t)1 << 40)) return fail(FDAS_ERR_INVALID_ARG, "n = %lld outside [1, 2^40]", (long long)n);
  if (n_harm < 1 || n_harm > 8) return fail(FDAS_ERR_INVALID_ARG, "n_harm = %d outside [1, 8]", (int)n_harm);
  if (nblocks < 0 || (nblocks > 0 && !h_blocks)) return fail(FDAS_ERR_INVALID_ARG, "bad block list");
  if (capacity < 0 || (capacity > 0 && !h_out)) return fail(FDAS_ERR_INVALID_ARG, "bad output buffer");
  const int64_t nblk = (n + kBlock - 1) / kBlock;
  for (int i = 0; i < nblocks; ++i)
    if (h_blocks[i] < 0 || h_blocks[i] >= nblk) return fail(FDAS_ERR_INVALID_ARG, "block %d outside the spectrum", h_blocks[i]);
  std::vector<char> mark((size_t)nblk, 0);
  for (int i = 0; i < nblocks; ++i) {
    const int64_t b = h_blocks[i];
    mark[(size_t)b] = 1;
    // block b holds columns [4096 b, 4096 b + 4095]; harmonic m of a signal
    // there raises the stretched sums at columns m j .. m j + m - 1
    for (int m = 2; m <= n_harm; ++m) {
      const int64_t lo = (int64_t)m * b * kBlock;
      const int64_t hi = std::min<int64_t>(n - 1, (int64_t)m * ((b + 1) * kBlock - 1) + m - 1);
      for (int64_t q = lo / kBlock; q <= hi / kBlock && q < nblk; ++q) mark[(size_t)q] = 1;
    }
  }
  int32_t cnt = 0;
  for (int64_t b = 0; b < nblk; ++b) {
    if (!mark[(size_t)b]) continue;
    if (cnt < capacity) h_out[cnt] = (int32_t)b;
    ++cnt;
  }
  *n_out = cnt;
  if (cnt > capacity) return fail(FDAS_ERR_CAPACITY, "closure of %d blocks > capacity %d", cnt, capacity);
  return ok();
}

fdas_status fdas_prescreen_init_params(uint64_t seed, float* h_theta) {
  if (!h_theta) return fail(FDAS_ERR_INVALID_ARG, "h_theta is NULL");
  // splitmix64 (Steele, Lea & Flood 2014): state += golden gamma, then mix
  uint64_t state = seed;
  auto next = [&state]() {
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  // uniform in [-1, 1) from the top 53 bits
  auto uni = [&next]() { return 2.0 * ((double)(next() >> 11) * (1.0 / 9007199254740992.0)) - 1.0; };
  constexpr int C = 32, K = 9;
  int o = 0;
  for (int l = 0; l < 4; ++l) {
    const int cin = l == 0 ? 1 : C;
    const double lim = std::sqrt(6.0 / (cin * K));  // He-uniform bound for ReLU layers
    for (int i = 0; i < C * cin * K; ++i) h_theta[o++] = (float)(lim * uni());
    for (int i = 0; i < C; ++i) h_theta[o++] = 0.0f;
  }
  for (int i = 0; i < C; ++i) h_theta[o++] = (float)(uni() / std::sqrt((double)C));
  h_theta[o++] = 0.0f;
  if (o != ps_param_count()) return fail(FDAS_ERR_DEVICE, "parameter layout mismatch (%d != %d)", o, ps_param_count());
  return ok();
}

fdas_status fdas_search_blocks(fdas_plan* p, const void* d_spectrum, int64_t n, float* d_fop, int64_t ld,
                               const int32_t* h_blocks, int32_t nblocks, fdas_cand* d_cands, int32_t* d_counts,
                               void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!d_spectrum || reinterpret_cast<uintptr_t>(d_spectrum) % 8 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "spectrum pointer is NULL or not 8-byte aligned");
  fdas_status st = check_fop_args(p, d_fop, n, ld);
  if (st != FDAS_OK) return st;
  if (!d_cands || reinterpret_cast<uintptr_t>(d_cands) % 16 != 0 || !d_counts)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffers are NULL or misaligned");
  if (nblocks < 0 || (nblocks > 0 && !h_blocks)) return fail(FDAS_ERR_INVALID_ARG, "bad block list");
  const int64_t nblk = (n + kBlock - 1) / kBlock;
  for (int i = 0; i < nblocks; ++i)
    if (h_blocks[i] < 0 || h_blocks[i] >= nblk) return fail(FDAS_ERR_INVALID_ARG, "block %d outside the spectrum", h_blocks[i]);
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool fast = !p->direct && p->desc.z_max == 42 && p->desc.hsum_index == FDAS_HSUM_STRETCH;
  if (!fast) {
    // other methods and index maps: the whole spectrum (a superset of the blocks)
    st = fdas_convolve(p, d_spectrum, n, d_fop, ld, stream);
    if (st == FDAS_OK) st = fdas_harmonic_sum(p, d_fop, n, ld, nullptr, d_cands, d_counts, stream);
    return st;
  }
  // columns to search (all FOP rows needed there), and the columns their
  // harmonic sums read as stretched sources (only the source rows needed)
  std::set<int64_t> search(h_blocks, h_blocks + nblocks);
  std::vector<char> full_block(nblk, 0), src_block(nblk, 0);
  const int nh = p->desc.n_harm;
  for (int64_t b : search) {
    const int64_t j0 = b * kBlock, j1 = std::min<int64_t>(n, j0 + kBlock) - 1;
    full_block[b] = 1;
    for (int k = 2; k <= nh; ++k) {
      // sources floor(j/k) and the neighbour floor(j/k) + 1 read for 4 columns at once
      const int64_t s0 = (j0 / 4 * 4) / k, s1 = std::min<int64_t>(n - 1, ((j1 / 4 * 4 + 3) / k) + 1);
      for (int64_t q = s0 / kBlock; q <= s1 / kBlock; ++q) src_block[q] = 1;
    }
  }
  // overlap-save chunks whose valid outputs touch a searched block (every
  // template) or only source blocks (the source rows)
  const OlsTables& ot = p->ols[p->ols_idx];
  const int slots = ols_slots(p, ot.geom.C);
  const int V = ot.geom.V;
  std::vector<int> chunks, src_chunks;
  const int64_t nchunks = (n + V - 1) / V;
  for (int64_t c = 0; c < nchunks; ++c) {
    const int64_t a = c * V, z = std::min<int64_t>(n, a + V) - 1;
    bool full = false, src = false;
    for (int64_t q = a / kBlock; q <= z / kBlock; ++q) {
      full = full || full_block[q] != 0;
      src = src || src_block[q] != 0;
    }
    if (full) chunks.push_back((int)c);
    else if (src) src_chunks.push_back((int)c);
  }
  int r_lo = 0, r_hi = -1;
  stretch_source_rows(p->desc.z_max, nh, &r_lo, &r_hi);
  // harmonic-sum tiles (1024 columns) of the searched blocks
  std::vector<int> tiles;
  const int tcols = harmsum_tile_columns();
  const int64_t ntiles = (n + tcols - 1) / tcols;
  for (int64_t b : search)
    for (int64_t t = b * (kBlock / tcols); t < (b + 1) * (kBlock / tcols) && t < ntiles; ++t) tiles.push_back((int)t);
  hipError_t e = hipSuccess;
  const size_t need = chunks.size() + src_chunks.size() + tiles.size() + 2;
  if ((int64_t)need > p->list_cap) {
    if (p->d_lists) (void)hipFree(p->d_lists);
    p->d_lists = nullptr;
    p->list_cap = 0;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_lists), need * sizeof(int))) != hipSuccess)
      return hip_fail(e, "allocating the block lists");
    p->list_cap = (int64_t)need;
  }
  std::vector<int> lists(chunks);
  lists.insert(lists.end(), src_chunks.begin(), src_chunks.end());
  lists.insert(lists.end(), tiles.begin(), tiles.end());
  // the lists are small and read by this call's kernels only: copy synchronously
  if (!lists.empty() &&
      ((e = hipStreamSynchronize(s)) != hipSuccess ||
       (e = hipMemcpy(p->d_lists, lists.data(), lists.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess))
    return hip_fail(e, "uploading the block lists");
  if (tiles.empty()) e = launch_fill_i32(d_counts, nh, 0, s);  // else the harmonic sum resets them
  if (e == hipSuccess && !chunks.empty())
    e = launch_ols_conv_list(static_cast<const float2*>(d_spectrum), n, d_fop, ld, ot, 0, p->rows, p->desc.z_max,
                             slots, p->d_lists, (int)chunks.size(), s);
  if (e == hipSuccess && !src_chunks.empty())
    e = launch_ols_conv_list(static_cast<const float2*>(d_spectrum), n, d_fop, ld, ot, r_lo, r_hi - r_lo + 1,
                             p->desc.z_max, slots, p->d_lists + chunks.size(), (int)src_chunks.size(), s);
  if (e == hipSuccess && !tiles.empty()) {
    HsWork wk{p->d_lists + chunks.size() + src_chunks.size(), (int)tiles.size(), p->d_hitrows, p->d_hitrow_count,
              p->tuning.emit_workgroups};
    e = launch_harmsum(d_fop, n, ld, p->desc.z_max, nh, p->d_ta, d_cands, p->desc.cand_capacity, d_counts, wk,
                       FDAS_HSUM_STRETCH, s);
  }
  if (e != hipSuccess) return hip_fail(e, "launching the block search");
  return ok();
}

fdas_status fdas_search_flagged(fdas_plan* p, const void* d_spectrum, int64_t n, float* d_fop, int64_t ld,
                                const float* d_logits, float threshold, fdas_cand* d_cands, int32_t* d_counts,
                                void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!d_spectrum || reinterpret_cast<uintptr_t>(d_spectrum) % 8 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "spectrum pointer is NULL or not 8-byte aligned");
  fdas_status st = check_fop_args(p, d_fop, n, ld);
  if (st != FDAS_OK) return st;
  if (!d_cands || reinterpret_cast<uintptr_t>(d_cands) % 16 != 0 || !d_counts)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffers are NULL or misaligned");
  if (!d_logits) {
    // the screen is disabled: the plain search
    st = fdas_convolve(p, d_spectrum, n, d_fop, ld, stream);
    if (st == FDAS_OK) st = fdas_harmonic_sum(p, d_fop, n, ld, nullptr, d_cands, d_counts, stream);
    return st;
  }
  if (reinterpret_cast<uintptr_t>(d_logits) % 4 != 0) return fail(FDAS_ERR_INVALID_ARG, "logits pointer is misaligned");
  const int64_t nblk = (n + kBlock - 1) / kBlock;
  if (nblk > kMaxSelBlocks)
    return fail(FDAS_ERR_INVALID_ARG, "n = %lld has more than %d blocks of %d bins", (long long)n, kMaxSelBlocks,
                kBlock);
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool fast = !p->direct && p->desc.z_max == 42 && p->desc.hsum_index == FDAS_HSUM_STRETCH;
  if (!fast) {
    // other methods and index maps: the whole spectrum (a superset of any selection)
    st = fdas_convolve(p, d_spectrum, n, d_fop, ld, stream);
    if (st == FDAS_OK) st = fdas_harmonic_sum(p, d_fop, n, ld, nullptr, d_cands, d_counts, stream);
    return st;
  }
  // lists sized for the whole spectrum: every chunk twice (searched, source
  // only), every tile, three counts
  const OlsTables& ot = p->ols[p->ols_idx];
  const int slots = ols_slots(p, ot.geom.C);
  const int V = ot.geom.V;
  const int tcols = harmsum_tile_columns();
  const int cap_c = (int)((n + V - 1) / V);
  const int cap_t = (int)((n + tcols - 1) / tcols);
  const int64_t need = 2 * (int64_t)cap_c + cap_t + 3;
  hipError_t e = hipSuccess;
  if (need > p->list_cap) {
    // an earlier call's kernels may still read the old lists
    if (p->d_lists && (e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "waiting for the stream");
    if (p->d_lists) (void)hipFree(p->d_lists);
    p->d_lists = nullptr;
    p->list_cap = 0;
    if ((e = hipMalloc(reinterpret_cast<void**>(&p->d_lists), need * sizeof(int))) != hipSuccess)
      return hip_fail(e, "allocating the block lists");
    p->list_cap = need;
  }
  const int nh = p->desc.n_harm;
  int* lists = p->d_lists;
  int* counts3 = lists + 2 * cap_c + cap_t;  // searched chunks, tiles, source-only chunks
  int r_lo = 0, r_hi = -1;
  stretch_source_rows(p->desc.z_max, nh, &r_lo, &r_hi);
  e = ps_search_lists(d_logits, threshold, n, (int)nblk, nh, V, tcols, lists, cap_c, cap_t, s);
  if (e == hipSuccess)
    e = launch_ols_conv_list(static_cast<const float2*>(d_spectrum), n, d_fop, ld, ot, 0, p->rows, p->desc.z_max,
                             slots, lists, cap_c, s, counts3);
  if (e == hipSuccess)
    e = launch_ols_conv_list(static_cast<const float2*>(d_spectrum), n, d_fop, ld, ot, r_lo, r_hi - r_lo + 1,
                             p->desc.z_max, slots, lists + cap_c + cap_t, cap_c, s, counts3 + 2);
  if (e == hipSuccess) {
    // every tile slot gets a workgroup; slots past the selection hold -1 and exit
    HsWork wk{lists + cap_c, cap_t, p->d_hitrows, p->d_hitrow_count, p->tuning.emit_workgroups};
    e = launch_harmsum(d_fop, n, ld, p->desc.z_max, nh, p->d_ta, d_cands, p->desc.cand_capacity, d_counts, wk,
                       FDAS_HSUM_STRETCH, s);
  }
  if (e != hipSuccess) return hip_fail(e, "launching the flagged-block search");
  return ok();
}

}  // extern "C"
