// Direct FIR correlation of the spectrum with every acceleration template on
// the matrix cores, fused with the power (Section 2.1.1, eq. (1): the
// time-domain FIR form, here as a Toeplitz-window x template contraction).
//
//   Y[j, z] = sum_d X[j + d] h_z[d],   FOP[z + z_max][j] = |Y[j, z]|^2.
//
// As a matrix product, row j of the window matrix is X[j + d] over the taps d
// and column z of the template matrix is h_z[d]; the window matrix is never
// formed: a workgroup stages its strip of X in LDS once and every MFMA operand
// is read from the strip at offset (row + tap).
//
// MFMA mapping (v_mfma_f32_16x16x4f32, one 16 x 16 FP32 output block,
// K = 4 real values = 2 complex taps per instruction):
//   rows    = 16 consecutive output bins;
//   columns = 8 templates x {Re Y, Im Y};
//   k       = (tap d, Re X), (d, Im X), (d + 1, Re X), (d + 1, Im X).
// With X = a + ib and h = c + is, Re Y += a c - b s and Im Y += a s + b c, so
// the packed template operand holds (c, -s) in the Re-column and (s, c) in the
// Im-column for the (Re X, Im X) pair of each tap; the plan packs it in lane
// order, 64 floats per tap pair.
//
// Templates are grouped by |z| in tiles of 8, and a tile only runs over the
// union of its members' supports [-P, P-1] (P = largest L/2 in the tile), so
// short templates do not pay for the 394-tap ones.  After the tap loop the
// lane holding Re Y and its neighbour holding Im Y swap values (DPP quad
// permutation), form |Y|^2, and store two bins each.
//
// Work split: a workgroup = 4 waves covers 512 consecutive bins; a wave owns
// 8 sub-tiles of 16 bins (8 independent accumulators keep the MFMA pipe full
// without waiting on one accumulator chain) and runs every template tile.

#include "fdas_internal.h"

namespace fdas {
namespace {

// Two adjacent FOP values stored non-temporally: the plane is written once and
// read back only after the whole convolution, so it should not stay in the
// caches (the same policy as the overlap-save kernel's stores).
__device__ __forceinline__ void store2_nt(float* dst, float a, float b) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = {a, b};
  __builtin_nontemporal_store(v, reinterpret_cast<f2v*>(dst));
}

constexpr int DW = 4;                 // waves per workgroup
constexpr int SUB = 8;                // 16-bin sub-tiles per wave
constexpr int WAVE_BINS = 16 * SUB;   // 128
constexpr int BLK_BINS = DW * WAVE_BINS;  // 512
constexpr int MAX_P = 296;            // L(64)/2, the widest template the plan allows

typedef float v4f __attribute__((ext_vector_type(4)));

// value of the neighbouring lane (lanes 2q and 2q+1 swap)
__device__ __forceinline__ float swap_pair(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

// tiles[g] = {P (tap pairs), first tap pair in Bpk, member count, P rounded up to 8};
// rows[g * 8 + t] = FOP row of member t.  Dynamic LDS: the X strip
// (2 * (BLK_BINS + 2 Pm + 16) floats) followed by one tile's template operand
// (64 * max padded pairs floats).
__global__ __launch_bounds__(DW * 64) void k_direct_conv(const float2* __restrict__ x, int64_t n,
                                                         float* __restrict__ fop, int64_t ld,
                                                         const float* __restrict__ Bpk,
                                                         const int4* __restrict__ tiles,
                                                         const int* __restrict__ rows, int ntiles, int Pm) {
  extern __shared__ float4 lds4[];
  float* xs = reinterpret_cast<float*>(lds4);
  const int tid = threadIdx.x;
  const int64_t jb = (int64_t)blockIdx.x * BLK_BINS;
  // strip X[jb - Pm + u], u < BLK_BINS + 2 Pm, plus 16 bins read (against
  // zero template values) by the padding pairs of a tile's last group of 8
  const int strip = BLK_BINS + 2 * Pm + 16;
  float* bs = xs + 2 * strip;  // strip is even: bs stays 16-byte aligned
  for (int u = tid; u < strip; u += DW * 64) {
    const int64_t idx = jb - Pm + u;
    const float2 v = (idx >= 0 && idx < n) ? x[idx] : make_float2(0.0f, 0.0f);
    xs[2 * u] = v.x;
    xs[2 * u + 1] = v.y;
  }

  const int lane = tid & 63;
  const int w = tid >> 6;
  const int m = lane & 15;  // A row (bin) / output column
  const int kk = lane >> 4; // A/B k index; output row group
  const int col = lane & 15;
  const int slot = col >> 1;
  const int c = col & 1;

  for (int g = 0; g < ntiles; ++g) {
    const int4 tg = tiles[g];
    const int P = tg.x;   // tap pairs of the tile's support
    const int P8 = tg.w;  // P rounded up to 8 (zero-padded in Bpk)
    {
      // stage the tile's template operand (P8 * 64 floats) in LDS
      const float4* __restrict__ src = reinterpret_cast<const float4*>(Bpk + (size_t)tg.y * 64);
      float4* dst = reinterpret_cast<float4*>(bs);
      __syncthreads();  // previous tile's operand no longer in use (and the strip is complete)
      for (int i = tid; i < P8 * 16; i += DW * 64) dst[i] = src[i];
      __syncthreads();
    }
    // this lane's A value of tap pair 0, sub-tile 0; pairs are 4 floats apart, sub-tiles 32
    const float* __restrict__ a = xs + 2 * (w * WAVE_BINS + m + Pm - P) + kk;
    const float* __restrict__ b = bs + lane;
    v4f acc[SUB];
#pragma unroll
    for (int s = 0; s < SUB; ++s) acc[s] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    for (int p = 0; p < P8; p += 8) {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float bv = b[64 * (p + u)];
#pragma unroll
        for (int s = 0; s < SUB; ++s)
          acc[s] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[32 * s + 4 * (p + u)], bv, acc[s], 0, 0, 0);
      }
    }
    const int row = slot < tg.z ? rows[g * 8 + slot] : -1;
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      float pw[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float o = swap_pair(acc[s][v]);
        pw[v] = acc[s][v] * acc[s][v] + o * o;
      }
      if (row >= 0) {
        // this lane stores bins j0 + 2c and j0 + 2c + 1 of its template
        const int64_t j = jb + w * WAVE_BINS + 16 * s + 4 * kk + 2 * c;
        float* dst = fop + (size_t)row * ld + j;
        const float p0 = c ? pw[2] : pw[0];
        const float p1 = c ? pw[3] : pw[1];
        if (j + 2 <= n) {
          store2_nt(dst, p0, p1);
        } else if (j < n) {
          __builtin_nontemporal_store(p0, dst);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split precision on the 16-bit matrix cores (v_mfma_f32_16x16x32_{f16,bf16}):
// every operand value v is carried as hi = round16(v), lo = round16(v - hi),
// and a product as hi*hi + hi*lo + lo*hi with FP32 accumulation (the lo*lo
// term, ~2^-22 of the product for FP16, is dropped).  One instruction takes
// 16 bins x 16 complex taps x 8 templates: K = 32 real values, lane group
// g = lane/16 holding taps 4g..4g+3 of the 16 as (Re, Im) pairs.  FP16 has a
// narrow exponent range, so the block's strip of X is scaled by 2^ex
// (largest |Re|, |Im| brought to about 2^14) and each template tile by a
// plan-chosen 2^eh; both scalings are exact and undone on the accumulator.

template <typename T>
struct Split16;

template <>
struct Split16<_Float16> {
  typedef _Float16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ unsigned short bits(float v) {
    const _Float16 h = (_Float16)v;
    return __builtin_bit_cast(unsigned short, h);
  }
  static __device__ __forceinline__ float value(unsigned short b) {
    return (float)__builtin_bit_cast(_Float16, b);
  }
  static __device__ __forceinline__ v4f mfma(const v8& a, const v8& b, const v4f& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <>
struct Split16<__bf16> {
  typedef __bf16 v8 __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ unsigned short bits(float v) {
    const __bf16 h = (__bf16)v;  // round to nearest even
    return __builtin_bit_cast(unsigned short, h);
  }
  static __device__ __forceinline__ float value(unsigned short b) {
    return __uint_as_float((unsigned)b << 16);
  }
  static __device__ __forceinline__ v4f mfma(const v8& a, const v8& b, const v4f& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// 8 16-bit values from 4 (possibly only 4-byte aligned) 32-bit LDS words
template <typename V8>
__device__ __forceinline__ V8 lds_v8(const unsigned* __restrict__ p) {
  uint4 u;
  u.x = p[0];
  u.y = p[1];
  u.z = p[2];
  u.w = p[3];
  return __builtin_bit_cast(V8, u);
}

// tiles[g] = {P, first 16-tap group in Bsp, member count, P rounded up to 8};
// Bsp holds per tile and 16-tap group 64 lanes x 8 hi values, then 64 x 8 lo
// values (2 KiB); tscale[g] = 2^-eh of the tile.  Dynamic LDS: hi and lo
// strips of X (2 x (BLK_BINS + 2 Pm + 16) words) and one tile's operand.
// Four waves per SIMD (at most 128 registers: the accumulators stay in VGPRs)
// keep the 16-bit matrix pipe busier than the compiler's default of three
// with AGPR accumulators (measured 1.67 against 1.85 ms on 2^22 bins).
template <typename T>
__global__ __launch_bounds__(DW * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_direct_conv_split(const float2* __restrict__ x, int64_t n,
                                                               float* __restrict__ fop, int64_t ld,
                                                               const uint4* __restrict__ Bsp,
                                                               const int4* __restrict__ tiles,
                                                               const float* __restrict__ tscale,
                                                               const int* __restrict__ rows, int ntiles, int Pm) {
  typedef Split16<T> S;
  typedef typename S::v8 v8;
  extern __shared__ uint4 lds_u4[];
  __shared__ unsigned s_max;
  unsigned* xhi = reinterpret_cast<unsigned*>(lds_u4);
  const int tid = threadIdx.x;
  const int64_t jb = (int64_t)blockIdx.x * BLK_BINS;
  const int strip = BLK_BINS + 2 * Pm + 16;  // even
  unsigned* xlo = xhi + strip;
  uint4* bs = reinterpret_cast<uint4*>(xlo + strip);
  if (tid == 0) s_max = 0u;
  __syncthreads();
  // largest |Re|, |Im| of the strip (bit patterns of non-negative floats order like integers)
  {
    float mx = 0.0f;
    for (int u = tid; u < strip; u += DW * 64) {
      const int64_t idx = jb - Pm + u;
      if (idx >= 0 && idx < n) {
        const float2 v = x[idx];
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
      }
    }
    atomicMax(&s_max, __float_as_uint(mx));
  }
  __syncthreads();
  int ex = 0;
  {
    const float mx = __uint_as_float(s_max);
    if (mx > 0.0f && mx < 3.0e38f) ex = 14 - ilogbf(mx);  // 2^14 <= max * 2^ex < 2^15
  }
  for (int u = tid; u < strip; u += DW * 64) {
    const int64_t idx = jb - Pm + u;
    const float2 v = (idx >= 0 && idx < n) ? x[idx] : make_float2(0.0f, 0.0f);
    const float re = ldexpf(v.x, ex), im = ldexpf(v.y, ex);
    const unsigned short hr = S::bits(re), hi_ = S::bits(im);
    const unsigned short lr = S::bits(re - S::value(hr)), li = S::bits(im - S::value(hi_));
    xhi[u] = (unsigned)hr | ((unsigned)hi_ << 16);
    xlo[u] = (unsigned)lr | ((unsigned)li << 16);
  }

  const int lane = tid & 63;
  const int w = tid >> 6;
  const int m = lane & 15;
  const int kg = lane >> 4;  // lane group: taps 4kg..4kg+3 of each 16
  const int col = lane & 15;
  const int slot = col >> 1;
  const int c = col & 1;

  for (int g = 0; g < ntiles; ++g) {
    const int4 tg = tiles[g];
    const int P = tg.x;
    const int groups16 = tg.w / 8;  // P8 pairs = 2 P8 taps = P8/8 groups of 16 taps
    {
      const uint4* __restrict__ src = Bsp + (size_t)tg.y * 128;  // 2 KiB = 128 uint4 per group, hi then lo
      __syncthreads();
      for (int i = tid; i < groups16 * 128; i += DW * 64) bs[i] = src[i];
      __syncthreads();
    }
    // strip word of this lane's first tap for group 0, sub-tile 0.  The A
    // operand of sub-tile s and tap group q starts at a0 + 16 (s + q): it
    // depends on s + q only, so a window of SUB operands slides along q, one
    // new (hi, lo) pair loaded per group (ring slot (s + q) % SUB, a
    // compile-time index inside the unrolled block of SUB groups).  Loading
    // the next group's operands one group ahead was slower (more registers,
    // two waves per SIMD instead of three).
    const int a0 = w * WAVE_BINS + m + Pm - P + 4 * kg;
    v4f acc[SUB];
#pragma unroll
    for (int s = 0; s < SUB; ++s) acc[s] = v4f{0.0f, 0.0f, 0.0f, 0.0f};
    v8 ah[SUB], al[SUB];
#pragma unroll
    for (int i = 0; i < SUB - 1; ++i) {
      ah[i] = lds_v8<v8>(xhi + a0 + 16 * i);
      al[i] = lds_v8<v8>(xlo + a0 + 16 * i);
    }
    for (int q0 = 0; q0 < groups16; q0 += SUB) {
#pragma unroll
      for (int dq = 0; dq < SUB; ++dq) {
        const int q = q0 + dq;
        if (q < groups16) {  // uniform
          ah[(dq + SUB - 1) % SUB] = lds_v8<v8>(xhi + a0 + 16 * (q + SUB - 1));
          al[(dq + SUB - 1) % SUB] = lds_v8<v8>(xlo + a0 + 16 * (q + SUB - 1));
          const v8 b_hi = __builtin_bit_cast(v8, bs[q * 128 + lane]);
          const v8 b_lo = __builtin_bit_cast(v8, bs[q * 128 + 64 + lane]);
#pragma unroll
          for (int s = 0; s < SUB; ++s) {
            const v8 a_hi = ah[(dq + s) % SUB];
            const v8 a_lo = al[(dq + s) % SUB];
            acc[s] = S::mfma(a_hi, b_hi, acc[s]);
            acc[s] = S::mfma(a_hi, b_lo, acc[s]);
            acc[s] = S::mfma(a_lo, b_hi, acc[s]);
          }
        }
      }
    }
    const float unscale = ldexpf(tscale[g], -ex);
    const int row = slot < tg.z ? rows[g * 8 + slot] : -1;
#pragma unroll
    for (int s = 0; s < SUB; ++s) {
      float pw[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float y = acc[s][v] * unscale;
        const float o = swap_pair(y);
        pw[v] = y * y + o * o;
      }
      if (row >= 0) {
        const int64_t j = jb + w * WAVE_BINS + 16 * s + 4 * kg + 2 * c;
        float* dst = fop + (size_t)row * ld + j;
        const float p0 = c ? pw[2] : pw[0];
        const float p1 = c ? pw[3] : pw[1];
        if (j + 2 <= n) {
          store2_nt(dst, p0, p1);
        } else if (j < n) {
          __builtin_nontemporal_store(p0, dst);
        }
      }
    }
  }
}

}  // namespace

int direct_block_bins() { return BLK_BINS; }
int direct_max_half_taps() { return MAX_P; }
size_t direct_lds_bytes(int P_max, int P8_max) {
  return sizeof(float) * (2 * (size_t)(BLK_BINS + 2 * P_max + 16) + 64 * (size_t)P8_max);
}

hipError_t launch_direct_conv_split(const float2* x, int64_t n, float* fop, int64_t ld, const DirectTables& t,
                                    bool bf16, hipStream_t s) {
  if (t.P_max > MAX_P || t.ntiles < 1 || n < 1 || !t.Bsp || !t.tscale) return hipErrorInvalidValue;
  const int64_t blocks = (n + BLK_BINS - 1) / BLK_BINS;
  const size_t lds = direct_lds_bytes(t.P_max, t.P8_max);
  const void* fn = bf16 ? reinterpret_cast<const void*>(k_direct_conv_split<__bf16>)
                        : reinterpret_cast<const void*>(k_direct_conv_split<_Float16>);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  if (bf16)
    hipLaunchKernelGGL(k_direct_conv_split<__bf16>, dim3((unsigned)blocks), dim3(DW * 64), lds, s, x, n, fop, ld,
                       t.Bsp, t.tiles, t.tscale, t.rows, t.ntiles, t.P_max);
  else
    hipLaunchKernelGGL(k_direct_conv_split<_Float16>, dim3((unsigned)blocks), dim3(DW * 64), lds, s, x, n, fop, ld,
                       t.Bsp, t.tiles, t.tscale, t.rows, t.ntiles, t.P_max);
  return hipGetLastError();
}

hipError_t launch_direct_conv(const float2* x, int64_t n, float* fop, int64_t ld, const DirectTables& t,
                              hipStream_t s) {
  if (t.P_max > MAX_P || t.ntiles < 1 || n < 1) return hipErrorInvalidValue;
  const int64_t blocks = (n + BLK_BINS - 1) / BLK_BINS;
  const size_t lds = direct_lds_bytes(t.P_max, t.P8_max);
  if (lds > 65536) {
    // above 64 KiB (templates wider than |z| = 42) the kernel must opt in
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_direct_conv),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_direct_conv, dim3((unsigned)blocks), dim3(DW * 64), lds, s, x, n, fop, ld, t.Bpk, t.tiles,
                     t.rows, t.ntiles, t.P_max);
  return hipGetLastError();
}

}  // namespace fdas
