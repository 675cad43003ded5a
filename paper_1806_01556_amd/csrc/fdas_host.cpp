// libfdas host side: plan creation, argument validation, kernel launches and
// candidate readback behind the C ABI of include/fdas.h.

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fdas_plan.h"

namespace fdas {

thread_local std::string g_err;

fdas_status fail(fdas_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

fdas_status ok() {
  g_err.clear();
  return FDAS_OK;
}

fdas_status hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) return fail(FDAS_ERR_OUT_OF_MEMORY, "%s: %s", what, hipGetErrorString(e));
  return fail(FDAS_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

void free_plan(fdas_plan* p) {
  if (!p) return;
  if (p->d_Bpk) (void)hipFree(p->d_Bpk);
  if (p->d_Bsp) (void)hipFree(p->d_Bsp);
  if (p->d_tscale) (void)hipFree(p->d_tscale);
  if (p->d_dtiles) (void)hipFree(p->d_dtiles);
  if (p->d_drows) (void)hipFree(p->d_drows);
  for (auto& t : p->ols) {
    if (t.H) (void)hipFree(t.H);
    if (t.tw1) (void)hipFree(t.tw1);
    if (t.tw2) (void)hipFree(t.tw2);
  }
  if (p->d_ta) (void)hipFree(p->d_ta);
  if (p->d_sort_a) (void)hipFree(p->d_sort_a);
  if (p->d_sort_b) (void)hipFree(p->d_sort_b);
  if (p->d_sort_hist) (void)hipFree(p->d_sort_hist);
  if (p->d_sort_totals) (void)hipFree(p->d_sort_totals);
  if (p->h_counts) (void)hipHostFree(p->h_counts);
  if (p->h_result) (void)hipHostFree(p->h_result);
  if (p->h_result_counts) (void)hipHostFree(p->h_result_counts);
  for (auto& kv : p->tile_orders) (void)hipFree(kv.second.first);
  if (p->d_hitrows) (void)hipFree(p->d_hitrows);
  if (p->d_hitrow_count) (void)hipFree(p->d_hitrow_count);
  if (p->d_lists) (void)hipFree(p->d_lists);
  free_batch(p);
  delete p;
}

template <typename T>
hipError_t upload(T** dst, const void* src, size_t bytes) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), bytes);
  if (e != hipSuccess) {
    *dst = nullptr;
    return e;
  }
  return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
}

fdas_status check_fop_args(const fdas_plan* p, const void* fop, int64_t n, int64_t ld) {
  if (!fop) return fail(FDAS_ERR_INVALID_ARG, "FOP pointer is NULL");
  if (reinterpret_cast<uintptr_t>(fop) % 16 != 0) return fail(FDAS_ERR_INVALID_ARG, "FOP pointer must be 16-byte aligned");
  if (n < 1 || n > p->desc.n_max)
    return fail(FDAS_ERR_INVALID_ARG, "n = %lld outside [1, n_max = %lld]", (long long)n, (long long)p->desc.n_max);
  if (ld < n) return fail(FDAS_ERR_INVALID_ARG, "ld = %lld < n = %lld", (long long)ld, (long long)n);
  if (ld % 4 != 0) return fail(FDAS_ERR_INVALID_ARG, "ld = %lld is not a multiple of 4", (long long)ld);
  return FDAS_OK;
}

void keep_top_k(const fdas_cand* sorted, const int* off, int nh, int top_k, std::vector<fdas_cand>& keep) {
  // each plane keeps its top_k powers (ties: lower z, then lower r), in (z, r) order
  for (int k = 0; k < nh; ++k) {
    std::vector<fdas_cand> v(sorted + off[k], sorted + off[k + 1]);
    if ((int)v.size() > top_k) {
      std::sort(v.begin(), v.end(), [](const fdas_cand& a, const fdas_cand& b) {
        if (a.power != b.power) return a.power > b.power;
        if (a.z != b.z) return a.z < b.z;
        return a.r < b.r;
      });
      v.resize(top_k);
      std::sort(v.begin(), v.end(), [](const fdas_cand& a, const fdas_cand& b) {
        if (a.z != b.z) return a.z < b.z;
        return a.r < b.r;
      });
    }
    keep.insert(keep.end(), v.begin(), v.end());
  }
}

// Device address of the static scratch array of fdas_harmonic_sum_noalloc,
// resolved once per device (at the first plan created on it, with the device
// current) and kept for the life of the process.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t resolve_noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  hipError_t e = harmsum_noalloc_scratch(&ptr);
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t ols_tables(fdas_plan* p, int C, const OlsTables** out) {
  const int idx = ols_index(C);
  if (idx < 0 || !ols_chunk_built(C)) return hipErrorInvalidValue;
  OlsTables& t = p->ols[idx];
  if (!t.H) {
    std::vector<std::vector<std::complex<double>>> bank;
    template_bank(p->desc.z_max, bank);
    OlsGeom g{C, p->L_max / 2, C - (p->L_max - 1)};
    std::vector<float> H, tw1, tw2;
    ols_spectra(bank, g.C, g.P, H);
    fft_twiddles(C, tw1, tw2);
    float2 *dH = nullptr, *d1 = nullptr, *d2 = nullptr;
    hipError_t e;
    if ((e = upload(&dH, H.data(), H.size() * sizeof(float))) != hipSuccess ||
        (e = upload(&d1, tw1.data(), tw1.size() * sizeof(float))) != hipSuccess ||
        (e = upload(&d2, tw2.data(), tw2.size() * sizeof(float))) != hipSuccess) {
      if (dH) (void)hipFree(dH);
      if (d1) (void)hipFree(d1);
      if (d2) (void)hipFree(d2);
      return e;
    }
    t.geom = g;
    t.H = dH;
    t.tw1 = d1;
    t.tw2 = d2;
  }
  *out = &t;
  return hipSuccess;
}

hipError_t tile_order_for(fdas_plan* p, int64_t n, const int** d_order, int* blocks, int cols) {
  const auto key = std::make_pair(n, cols);
  auto it = p->tile_orders.find(key);
  if (it == p->tile_orders.end()) {
    std::vector<int> order;
    harmsum_tile_order(n, order, cols);
    int* d = nullptr;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&d), order.size() * sizeof(int));
    if (e == hipSuccess) e = hipMemcpy(d, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      if (d) (void)hipFree(d);
      return e;
    }
    it = p->tile_orders.emplace(key, std::make_pair(d, (int)order.size())).first;
  }
  *d_order = it->second.first;
  *blocks = it->second.second;
  return hipSuccess;
}

}  // namespace fdas

using namespace fdas;

extern "C" {

void fdas_plan_desc_default(fdas_plan_desc* d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->struct_size = (int32_t)sizeof(fdas_plan_desc);
  d->z_max = 42;
  d->n_max = (int64_t)1 << 22;
  d->n_harm = 8;
  d->cand_capacity = 65536;
  d->p_fa = 1e-6;
  d->top_k = 0;
  d->method = FDAS_CONV_AUTO;
  d->precision = FDAS_PREC_FP32;
  d->hsum_index = FDAS_HSUM_STRETCH;
  d->ols_chunk = 0;
  d->device = 0;
}

const char* fdas_last_error(void) { return g_err.c_str(); }

int32_t fdas_abi_version(void) { return FDAS_ABI_VERSION; }

fdas_status fdas_template_taps(int32_t z, double* taps, int32_t capacity, int32_t* n_taps) {
  if (z < -64 || z > 64) return fail(FDAS_ERR_INVALID_ARG, "|z| = %d > 64", (int)z);
  const int L = fdas::tap_count(z);
  if (n_taps) *n_taps = L;
  if (!taps) return fail(FDAS_ERR_INVALID_ARG, "taps pointer is NULL");
  if (capacity < L) return fail(FDAS_ERR_INVALID_ARG, "capacity %d < %d taps", (int)capacity, L);
  std::vector<std::complex<double>> h;
  fdas::template_taps(z, h);
  for (int t = 0; t < L; ++t) {
    taps[2 * t] = h[t].real();
    taps[2 * t + 1] = h[t].imag();
  }
  return ok();
}

fdas_status fdas_thresholds(int32_t n_harm, double p_fa, double* out) {
  if (n_harm < 1 || n_harm > 8) return fail(FDAS_ERR_INVALID_ARG, "n_harm = %d outside [1, 8]", (int)n_harm);
  if (!(p_fa > 0.0 && p_fa < 1.0)) return fail(FDAS_ERR_INVALID_ARG, "p_fa must lie in (0, 1)");
  if (!out) return fail(FDAS_ERR_INVALID_ARG, "out pointer is NULL");
  for (int k = 1; k <= n_harm; ++k) out[k - 1] = fdas::erlang_threshold(k, p_fa);
  return ok();
}

fdas_status fdas_plan_create(const fdas_plan_desc* desc, fdas_plan** out) {
  if (!out) return fail(FDAS_ERR_INVALID_ARG, "out pointer is NULL");
  *out = nullptr;
  if (!desc) return fail(FDAS_ERR_INVALID_ARG, "descriptor is NULL");
  if (desc->struct_size != (int32_t)sizeof(fdas_plan_desc))
    return fail(FDAS_ERR_INVALID_ARG, "struct_size %d != %d (header/library mismatch)", (int)desc->struct_size,
                (int)sizeof(fdas_plan_desc));
  if (desc->z_max < 0 || desc->z_max > 64) return fail(FDAS_ERR_INVALID_ARG, "z_max = %d outside [0, 64]", (int)desc->z_max);
  if (desc->n_max < 1 || desc->n_max > ((int64_t)1 << 30))
    return fail(FDAS_ERR_INVALID_ARG, "n_max = %lld outside [1, 2^30]", (long long)desc->n_max);
  if ((int64_t)(2 * desc->z_max + 1) * desc->n_max > (int64_t)INT32_MAX)
    return fail(FDAS_ERR_INVALID_ARG, "(2*z_max+1) * n_max = %lld: per-plane candidate counts must stay below 2^31",
                (long long)(2 * desc->z_max + 1) * (long long)desc->n_max);
  if (desc->n_harm < 1 || desc->n_harm > 8) return fail(FDAS_ERR_INVALID_ARG, "n_harm = %d outside [1, 8]", (int)desc->n_harm);
  if (desc->cand_capacity < 1 || desc->cand_capacity > (1 << 22))
    return fail(FDAS_ERR_INVALID_ARG, "cand_capacity = %d outside [1, 2^22]", (int)desc->cand_capacity);
  if (!(desc->p_fa > 0.0 && desc->p_fa < 1.0)) return fail(FDAS_ERR_INVALID_ARG, "p_fa must lie in (0, 1)");
  if (desc->top_k < 0) return fail(FDAS_ERR_INVALID_ARG, "top_k < 0");
  if (desc->method != FDAS_CONV_AUTO && desc->method != FDAS_CONV_OLS_FFT && desc->method != FDAS_CONV_DIRECT_MFMA)
    return fail(FDAS_ERR_INVALID_ARG, "unknown method %d", (int)desc->method);
  if (desc->precision != FDAS_PREC_FP32 && desc->precision != FDAS_PREC_SPLIT_FP16 &&
      desc->precision != FDAS_PREC_SPLIT_BF16)
    return fail(FDAS_ERR_INVALID_ARG, "unknown precision %d", (int)desc->precision);
  if (desc->precision != FDAS_PREC_FP32 && desc->method != FDAS_CONV_DIRECT_MFMA)
    return fail(FDAS_ERR_INVALID_ARG, "split precisions apply to the direct method only");
  if (desc->hsum_index != FDAS_HSUM_STRETCH && desc->hsum_index != FDAS_HSUM_FUNDAMENTAL &&
      desc->hsum_index != FDAS_HSUM_HIGHEST)
    return fail(FDAS_ERR_INVALID_ARG, "unknown hsum_index %d", (int)desc->hsum_index);
  if (desc->ols_chunk != 0 && !fdas::ols_chunk_built(desc->ols_chunk))
    return fail(FDAS_ERR_UNSUPPORTED, "ols_chunk %d: the built chunk lengths are 2048, 4096 and 8192",
                (int)desc->ols_chunk);
  if (desc->ols_chunk != 0 && desc->ols_chunk - (fdas::tap_count(desc->z_max) - 1) < 1024)
    return fail(FDAS_ERR_INVALID_ARG, "ols_chunk %d leaves fewer than 1024 valid outputs for %d-tap templates",
                (int)desc->ols_chunk, fdas::tap_count(desc->z_max));

  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) return fail(FDAS_ERR_NO_DEVICE, "no HIP device (%s)", hipGetErrorString(e));
  if (desc->device < 0 || desc->device >= ndev)
    return fail(FDAS_ERR_NO_DEVICE, "device %d outside [0, %d)", (int)desc->device, ndev);

  fdas_plan* p = new (std::nothrow) fdas_plan();
  if (!p) return fail(FDAS_ERR_OUT_OF_MEMORY, "host allocation of the plan failed");
  p->desc = *desc;
  p->device = desc->device;
  p->rows = 2 * desc->z_max + 1;
  p->L_max = fdas::tap_count(desc->z_max);
  p->ols_idx = fdas::ols_index(desc->ols_chunk != 0 ? desc->ols_chunk : fdas::kOlsC);

  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) {
    free_plan(p);
    return hip_fail(dg.err, "hipSetDevice");
  }
  {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
      p->cus = cus;
  }
  if ((e = fdas::resolve_noalloc_scratch(p->device)) != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "resolving the static scratch address");
  }

  std::vector<std::vector<std::complex<double>>> bank;
  fdas::template_bank(desc->z_max, bank);
  p->direct = desc->method == FDAS_CONV_DIRECT_MFMA;
  std::vector<float> Bpk, tscale;
  std::vector<uint16_t> Bsp;
  std::vector<int> dtiles, drows;
  if (p->direct && desc->precision != FDAS_PREC_FP32) {
    fdas::direct_pack_split(bank, desc->z_max, desc->precision == FDAS_PREC_SPLIT_BF16, Bsp, tscale, dtiles, drows,
                            &p->dP_max, &p->dP8_max);
    p->dtiles = (int)dtiles.size() / 4;
  } else if (p->direct) {
    fdas::direct_pack(bank, desc->z_max, Bpk, dtiles, drows, &p->dP_max, &p->dP8_max);
    p->dtiles = (int)dtiles.size() / 4;
  }
  p->h_ta.resize((size_t)desc->n_harm * p->rows);
  for (int k = 1; k <= desc->n_harm; ++k) {
    const float t = (float)fdas::erlang_threshold(k, desc->p_fa);
    for (int r = 0; r < p->rows; ++r) p->h_ta[(size_t)(k - 1) * p->rows + r] = t;
  }

  if (p->direct && desc->precision != FDAS_PREC_FP32) {
    if ((e = upload(&p->d_Bsp, Bsp.data(), Bsp.size() * sizeof(uint16_t))) != hipSuccess ||
        (e = upload(&p->d_tscale, tscale.data(), tscale.size() * sizeof(float))) != hipSuccess ||
        (e = upload(&p->d_dtiles, dtiles.data(), dtiles.size() * sizeof(int))) != hipSuccess ||
        (e = upload(&p->d_drows, drows.data(), drows.size() * sizeof(int))) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "uploading the split direct-method template operand");
    }
  } else if (p->direct) {
    if ((e = upload(&p->d_Bpk, Bpk.data(), Bpk.size() * sizeof(float))) != hipSuccess ||
        (e = upload(&p->d_dtiles, dtiles.data(), dtiles.size() * sizeof(int))) != hipSuccess ||
        (e = upload(&p->d_drows, drows.data(), drows.size() * sizeof(int))) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "uploading the direct-method template operand");
    }
  } else {
    const fdas::OlsTables* t = nullptr;
    if ((e = fdas::ols_tables(p, desc->ols_chunk ? desc->ols_chunk : fdas::kOlsC, &t)) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "uploading the overlap-save template spectra");
    }
  }
  if ((e = upload(&p->d_ta, p->h_ta.data(), p->h_ta.size() * sizeof(float))) != hipSuccess) {
    free_plan(p);
    return hip_fail(e, "uploading plan tables");
  }
  {
    const size_t total = (size_t)desc->n_harm * desc->cand_capacity;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < desc->n_max) ++bits;
    const size_t tiles = (size_t)fdas::sort_tile_count((int)total);
    const size_t passes = (size_t)fdas::sort_passes(p->rows, bits);
    if ((e = hipMalloc(&p->d_sort_a, total * sizeof(fdas_cand))) != hipSuccess ||
        (e = hipMalloc(&p->d_sort_b, total * sizeof(fdas_cand))) != hipSuccess ||
        (e = hipMalloc(&p->d_sort_hist, 256 * tiles * sizeof(int))) != hipSuccess ||
        (e = hipMalloc(&p->d_sort_totals, 256 * passes * sizeof(int))) != hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&p->h_counts), 8 * sizeof(int32_t), 0)) != hipSuccess ||
        (e = hipMalloc(&p->d_hitrows, (size_t)((desc->n_max + 3) / 4) * sizeof(int4))) != hipSuccess ||
        (e = hipMalloc(&p->d_hitrow_count, sizeof(int32_t))) != hipSuccess) {
      free_plan(p);
      return hip_fail(e, "allocating the candidate sort workspace");
    }
    p->bits_r = bits;
  }
  *out = p;
  return ok();
}

fdas_status fdas_plan_destroy(fdas_plan* plan) {
  if (!plan) return ok();
  DeviceGuard dg(plan->device);
  (void)hipDeviceSynchronize();
  free_plan(plan);
  return ok();
}

fdas_status fdas_convolve(fdas_plan* p, const void* d_spectrum, int64_t n, float* d_fop, int64_t ld, void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!d_spectrum) return fail(FDAS_ERR_INVALID_ARG, "spectrum pointer is NULL");
  if (reinterpret_cast<uintptr_t>(d_spectrum) % 8 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "spectrum pointer must be 8-byte aligned");
  fdas_status st = check_fop_args(p, d_fop, n, ld);
  if (st != FDAS_OK) return st;
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipError_t e;
  if (p->direct) {
    const fdas::DirectTables t{p->d_Bpk, p->d_dtiles, p->d_drows, p->dtiles, p->dP_max, p->dP8_max,
                               p->d_Bsp, p->d_tscale};
    if (p->desc.precision == FDAS_PREC_FP32)
      e = fdas::launch_direct_conv(static_cast<const float2*>(d_spectrum), n, d_fop, ld, t,
                                   static_cast<hipStream_t>(stream));
    else
      e = fdas::launch_direct_conv_split(static_cast<const float2*>(d_spectrum), n, d_fop, ld, t,
                                         p->desc.precision == FDAS_PREC_SPLIT_BF16, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "launching the direct correlation");
  } else {
    const fdas::OlsTables& t = p->ols[p->ols_idx];
    e = fdas::launch_ols_conv(static_cast<const float2*>(d_spectrum), n, d_fop, ld, t, p->rows,
                              fdas::ols_slots(p, t.geom.C), static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return hip_fail(e, "launching the overlap-save convolution");
  }
  return ok();
}

fdas_status fdas_harmonic_sum(fdas_plan* p, const float* d_fop, int64_t n, int64_t ld, const float* d_ta,
                              fdas_cand* d_cands, int32_t* d_counts, void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  fdas_status st = check_fop_args(p, d_fop, n, ld);
  if (st != FDAS_OK) return st;
  if (!d_cands) return fail(FDAS_ERR_INVALID_ARG, "candidate buffer is NULL");
  if (reinterpret_cast<uintptr_t>(d_cands) % 16 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffer must be 16-byte aligned");
  if (!d_counts) return fail(FDAS_ERR_INVALID_ARG, "count buffer is NULL");
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // workgroup -> column-tile order of the 85-row kernel, built once per spectrum length
  const int* d_order = nullptr;
  int order_blocks = 0;
  {
    hipError_t e0 = fdas::tile_order_for(p, n, &d_order, &order_blocks);
    if (e0 != hipSuccess) return hip_fail(e0, "uploading the harmonic-sum tile order");
  }
  hipError_t e;
  fdas::HsWork wk{d_order, order_blocks, p->d_hitrows, p->d_hitrow_count, p->tuning.emit_workgroups};
  e = fdas::launch_harmsum(d_fop, n, ld, p->desc.z_max, p->desc.n_harm, d_ta ? d_ta : p->d_ta, d_cands,
                           p->desc.cand_capacity, d_counts, wk, p->desc.hsum_index, s);
  if (e != hipSuccess) return hip_fail(e, "launching the harmonic sum");
  return ok();
}

fdas_status fdas_harmonic_sum_noalloc(fdas_plan* p, const float* d_fop, int64_t n, int64_t ld, const float* d_ta,
                                      fdas_cand* d_cands, int32_t* d_counts, void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  fdas_status st = check_fop_args(p, d_fop, n, ld);
  if (st != FDAS_OK) return st;
  if (n > fdas::harmsum_noalloc_max_n())
    return fail(FDAS_ERR_INVALID_ARG, "n = %lld exceeds the %lld bins the static scratch of the allocation-free "
                "harmonic sum holds", (long long)n, (long long)fdas::harmsum_noalloc_max_n());
  if (!d_cands) return fail(FDAS_ERR_INVALID_ARG, "candidate buffer is NULL");
  if (reinterpret_cast<uintptr_t>(d_cands) % 16 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffer must be 16-byte aligned");
  if (!d_counts) return fail(FDAS_ERR_INVALID_ARG, "count buffer is NULL");
  void* scr = fdas::noalloc_scratch(p->device);
  if (!scr) return fail(FDAS_ERR_DEVICE, "static scratch address of device %d was not resolved", p->device);
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipError_t e = fdas::launch_harmsum_noalloc(d_fop, n, ld, p->desc.z_max, p->desc.n_harm, d_ta ? d_ta : p->d_ta,
                                              d_cands, p->desc.cand_capacity, d_counts, scr,
                                              p->tuning.emit_workgroups, p->desc.hsum_index,
                                              static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "launching the allocation-free harmonic sum");
  return ok();
}

fdas_status fdas_candidates(fdas_plan* p, const fdas_cand* d_cands, const int32_t* d_counts, fdas_cand* h_out,
                            int64_t h_capacity, int64_t* h_n, int32_t* h_counts, void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!d_cands || !d_counts) return fail(FDAS_ERR_INVALID_ARG, "device candidate buffers are NULL");
  if (reinterpret_cast<uintptr_t>(d_cands) % 16 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffer must be 16-byte aligned");
  if (!h_n) return fail(FDAS_ERR_INVALID_ARG, "h_n is NULL");
  if (h_capacity < 0 || (h_capacity > 0 && !h_out)) return fail(FDAS_ERR_INVALID_ARG, "bad host output buffer");
  *h_n = 0;
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nh = p->desc.n_harm;
  const int cap = p->desc.cand_capacity;
  // order on the device first (sizes come from the device counts), then one
  // wait for the counts, then the copy of the ordered records
  fdas_cand* sorted = nullptr;
  hipError_t e = fdas::launch_sort_candidates(d_cands, cap, nh, d_counts, p->rows, p->desc.z_max, p->bits_r,
                                              p->d_sort_a, p->d_sort_b, p->d_sort_hist, p->d_sort_totals, &sorted, s);
  if (e != hipSuccess) return hip_fail(e, "ordering candidates");
  int32_t* counts = p->h_counts;
  e = hipMemcpyAsync(counts, d_counts, nh * sizeof(int32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading candidate counts");
  if (h_counts) std::copy(counts, counts + nh, h_counts);
  bool overflow = false;
  int off[9] = {0};
  for (int k = 0; k < nh; ++k) {
    if (counts[k] < 0) return fail(FDAS_ERR_DEVICE, "negative candidate count");
    if (counts[k] > cap) overflow = true;
    off[k + 1] = off[k] + std::min(counts[k], cap);
  }
  int total = off[nh];
  const fdas_cand* src = sorted;
  if (p->desc.top_k > 0) {
    // paper mode (Table 1's N_cand): each plane keeps its top_k powers (ties:
    // lower z, then lower r), selected on the device into the other buffer
    fdas_cand* kept = sorted == p->d_sort_a ? p->d_sort_b : p->d_sort_a;
    e = fdas::launch_topk(sorted, cap, nh, d_counts, p->desc.top_k, kept, s);
    if (e != hipSuccess) return hip_fail(e, "selecting the top candidates");
    src = kept;
    total = 0;
    for (int k = 0; k < nh; ++k) total += std::min(off[k + 1] - off[k], p->desc.top_k);
  }
  const int64_t nw = std::min<int64_t>(total, h_capacity);
  if (nw > 0) e = hipMemcpyAsync(h_out, src, (size_t)nw * sizeof(fdas_cand), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading candidates");
  *h_n = nw;
  if (overflow) return fail(FDAS_ERR_CAPACITY, "a device candidate list overflowed (counts are exact)");
  if (nw < total) return fail(FDAS_ERR_CAPACITY, "h_capacity %lld < %d candidates", (long long)h_capacity, total);
  return ok();
}

fdas_status fdas_candidates_mapped(fdas_plan* p, const fdas_cand* d_cands, const int32_t* d_counts,
                                   const fdas_cand** h_view, int64_t* h_n, int32_t* h_counts, void* stream) {
  if (!p) return fail(FDAS_ERR_INVALID_ARG, "plan is NULL");
  if (!d_cands || !d_counts) return fail(FDAS_ERR_INVALID_ARG, "device candidate buffers are NULL");
  if (reinterpret_cast<uintptr_t>(d_cands) % 16 != 0)
    return fail(FDAS_ERR_INVALID_ARG, "candidate buffer must be 16-byte aligned");
  if (!h_view || !h_n) return fail(FDAS_ERR_INVALID_ARG, "h_view or h_n is NULL");
  *h_view = nullptr;
  *h_n = 0;
  DeviceGuard dg(p->device);
  if (dg.err != hipSuccess) return hip_fail(dg.err, "hipSetDevice");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nh = p->desc.n_harm;
  const int cap = p->desc.cand_capacity;
  hipError_t e = hipSuccess;
  if (!p->h_result &&
      (e = hipHostMalloc(reinterpret_cast<void**>(&p->h_result), (size_t)nh * cap * sizeof(fdas_cand), 0)) != hipSuccess) {
    p->h_result = nullptr;
    return hip_fail(e, "allocating the page-locked result buffer");
  }
  if (!p->h_result_counts &&
      (e = hipHostMalloc(reinterpret_cast<void**>(&p->h_result_counts), 8 * sizeof(int32_t), 0)) != hipSuccess) {
    p->h_result_counts = nullptr;
    return hip_fail(e, "allocating the page-locked result counts");
  }
  void* d_res = nullptr;
  void* d_rc = nullptr;
  if ((e = hipHostGetDevicePointer(&d_res, p->h_result, 0)) != hipSuccess ||
      (e = hipHostGetDevicePointer(&d_rc, p->h_result_counts, 0)) != hipSuccess)
    return hip_fail(e, "mapping the result buffer");
  fdas_cand* sorted = nullptr;
  const int keep = p->desc.top_k > 0 ? std::min(p->desc.top_k, cap) : 0;
  e = fdas::launch_sort_candidates(d_cands, cap, nh, d_counts, p->rows, p->desc.z_max, p->bits_r, p->d_sort_a,
                                   p->d_sort_b, p->d_sort_hist, p->d_sort_totals, &sorted, s);
  if (e == hipSuccess && keep > 0) {
    // paper mode: the top-k selection on the device, into the other buffer
    fdas_cand* kept = sorted == p->d_sort_a ? p->d_sort_b : p->d_sort_a;
    e = fdas::launch_topk(sorted, cap, nh, d_counts, keep, kept, s);
    sorted = kept;
  }
  if (e == hipSuccess)
    e = fdas::launch_copy_out(sorted, cap, nh, d_counts, nh * cap, static_cast<fdas_cand*>(d_res),
                              static_cast<int32_t*>(d_rc), s, keep);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "ordering and reading candidates");
  const int32_t* counts = p->h_result_counts;
  if (h_counts) std::copy(counts, counts + nh, h_counts);
  bool overflow = false;
  int64_t total = 0;
  for (int k = 0; k < nh; ++k) {
    if (counts[k] < 0) return fail(FDAS_ERR_DEVICE, "negative candidate count");
    if (counts[k] > cap) overflow = true;
    total += keep > 0 ? std::min(std::min(counts[k], cap), keep) : std::min(counts[k], cap);
  }
  *h_view = p->h_result;
  *h_n = total;
  if (overflow) return fail(FDAS_ERR_CAPACITY, "a device candidate list overflowed (counts are exact)");
  return ok();
}

}  // extern "C"
