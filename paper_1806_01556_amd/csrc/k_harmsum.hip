// Harmonic summing with threshold detection and candidate compaction
// (Section 2.2, Algorithm 1), all harmonic planes at once without storing
// them (the MultipleHP organisation of Section 2.2).
//
//   HP_1(i, j) = FOP(i, j)
//   HP_k(i, j) = HP_{k-1}(i, j) + FOP(trunc(i/k), floor(j/k)),  k = 2..NH
//   a cell with HP_k(i, j) > TA(k, i) is appended to list k.
//
// Each thread owns 4 adjacent columns j0..j0+3 (one 16-byte load per row of
// the unstretched plane) and walks all rows; for k >= 2 the 4 columns read at
// most two adjacent source columns (floor(j/k) spans <= 2 values when
// k >= 2), fetched once per change of the source row trunc(i/k) and kept in
// registers across the k rows that share it.  Sums are FP32 in k order (no
// reassociation), so results are bit-identical to a sequential FP32 sum.
// Candidates are appended with one atomic per plane per hit; the compiler's
// wave-level atomic aggregation combines hits of a wave.

#include "fdas_internal.h"

namespace fdas {
namespace {

constexpr int HS_THREADS = 256;

__device__ __forceinline__ void emit(int k, int i, int j, float p, fdas_cand* __restrict__ cands, int cap,
                                     int32_t* __restrict__ counts) {
  const int slot = atomicAdd(&counts[k - 1], 1);
  if (slot < cap) {
    int4 rec = make_int4(k, i, j, __float_as_int(p));
    *reinterpret_cast<int4*>(cands + (size_t)(k - 1) * cap + slot) = rec;
  }
}

template <int NH>
__global__ __launch_bounds__(HS_THREADS) void k_harmsum(const float* __restrict__ fop, int64_t ld, int n,
                                                        int z_max, const float* __restrict__ ta,
                                                        fdas_cand* __restrict__ cands, int cap,
                                                        int32_t* __restrict__ counts) {
  const int64_t g = (int64_t)blockIdx.x * HS_THREADS + threadIdx.x;
  const int64_t j0l = g * 4;
  if (j0l >= n) return;
  const int j0 = (int)j0l;
  const bool full = j0 + 4 <= n;
  const int rows = 2 * z_max + 1;

  int lo[NH + 1], hi[NH + 1];
  bool selhi[NH + 1][4];
#pragma unroll
  for (int m = 2; m <= NH; ++m) {
    lo[m] = j0 / m;
    hi[m] = min(lo[m] + 1, n - 1);
#pragma unroll
    for (int a = 0; a < 4; ++a) selhi[m][a] = ((j0 + a) / m) != lo[m];
  }
  float cache[NH + 1][4];
#pragma unroll
  for (int m = 0; m <= NH; ++m)
#pragma unroll
    for (int a = 0; a < 4; ++a) cache[m][a] = 0.0f;

  for (int r = 0; r < rows; ++r) {
    const int i = r - z_max;
    const float* row = fop + (size_t)r * ld;
    float hp[4];
    if (full) {
      const float4 q = *reinterpret_cast<const float4*>(row + j0);
      hp[0] = q.x;
      hp[1] = q.y;
      hp[2] = q.z;
      hp[3] = q.w;
    } else {
#pragma unroll
      for (int a = 0; a < 4; ++a) hp[a] = (j0 + a < n) ? row[j0 + a] : 0.0f;
    }
    {
      const float t = ta[r];
#pragma unroll
      for (int a = 0; a < 4; ++a)
        if (hp[a] > t && j0 + a < n) emit(1, i, j0 + a, hp[a], cands, cap, counts);
    }
#pragma unroll
    for (int m = 2; m <= NH; ++m) {
      const int si = i / m;  // C division: truncation toward zero
      if (r == 0 || si != (i - 1) / m) {
        const float* src = fop + (size_t)(si + z_max) * ld;
        const float vl = src[lo[m]];
        const float vh = src[hi[m]];
#pragma unroll
        for (int a = 0; a < 4; ++a) cache[m][a] = selhi[m][a] ? vh : vl;
      }
      const float t = ta[(m - 1) * rows + r];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        hp[a] = hp[a] + cache[m][a];
        if (hp[a] > t && j0 + a < n) emit(m, i, j0 + a, hp[a], cands, cap, counts);
      }
    }
  }
}

__global__ void k_fill_i32(int32_t* p, int count, int32_t value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

}  // namespace

hipError_t launch_harmsum(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm, const float* ta,
                          fdas_cand* cands, int cap, int32_t* counts, hipStream_t s) {
  const int64_t groups = (n + 3) / 4;
  const unsigned blocks = (unsigned)((groups + HS_THREADS - 1) / HS_THREADS);
  const int nn = (int)n;
  switch (n_harm) {
#define FDAS_HS_CASE(NH)                                                                                 \
  case NH:                                                                                               \
    hipLaunchKernelGGL(k_harmsum<NH>, dim3(blocks), dim3(HS_THREADS), 0, s, fop, ld, nn, z_max, ta, cands, \
                       cap, counts);                                                                     \
    break;
    FDAS_HS_CASE(1)
    FDAS_HS_CASE(2)
    FDAS_HS_CASE(3)
    FDAS_HS_CASE(4)
    FDAS_HS_CASE(5)
    FDAS_HS_CASE(6)
    FDAS_HS_CASE(7)
    FDAS_HS_CASE(8)
#undef FDAS_HS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

}  // namespace fdas
