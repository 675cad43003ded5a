// Overlap-save FFT correlation of a complex spectrum with every acceleration
// template, fused with the power and the discard of the overlap
// (Section 2.1.2 overlap-save FDFIR, eq. (2); power as in Section 2.2).
//
// One workgroup = one chunk of C input bins (C = 2048, 4096 or 8192; the
// chunk length N_OLS-FT is the design parameter of Section 2.1.2) and a group
// of templates:
//   chunk c covers outputs j in [c*V, c*V + V), V = C - (L_max - 1), and reads
//   X[c*V - P + t], t in [0, C), P = L_max/2, zero outside [0, n).
//   F = FFT(chunk) once (shared by all templates of the group, as the
//   area-efficient AOLS design of Section 2.1.3 transforms the input once),
//   then per template: y = IFFT(F * H_z), |y|^2 of the first V outputs -> FOP.
//   H_z = (1/C) * sum_t g_z[t] e^{+2 pi i t k / C} with g_z the template placed
//   at t = P + d, so y[s] = sum_d X[c*V + s + d] h_z[d] (centred correlation).
//
// A workgroup has NT = C/16 threads of 16 points; thread t holds x[t + NT r]
// in register r.  The C-point FFT is C = 16 * M: a 16-point DFT over r in
// registers, twiddle w_C^(nb t), then an M-point DFT over t for each of the 16
// rows nb, split again into 16-point DFTs and a last factor:
//   C = 4096: 16 x 16 x 16 (three radix-16 passes, two LDS transposes);
//   C = 2048: 16 x 16 x 8  (the last pass two 8-point DFTs per thread);
//   C = 8192: 16 x 16 x 16 x 2 (the 32-point last factor as radix 16, a
//             twiddle w32^(p c0), then radix 2; three LDS transposes).
// In every case the output element X[t + NT r] ends in register r of thread
// t, the layout of the input, so the forward result F stays in registers for
// every template and the inverse transform is the same code.  LDS row strides
// and the XOR swizzle (C = 4096) put the 32 lanes of every half-wave access on
// distinct banks.  No packed-FP32 instructions are written here (the build
// disables them).

#include <algorithm>

#include "fdas_internal.h"
#include "fft16.h"

namespace fdas {
namespace {

using namespace fft;

template <int C>
struct Shape;
template <>
struct Shape<2048> {
  static constexpr int NT = 128;             // threads
  static constexpr int TW2 = 8;              // columns c of the second twiddle table, w128^(q c)
  static constexpr int RS1 = 136;            // buffer 1: 16 rows of 128, padded
  static constexpr int B2 = 16 * RS1;        // buffer 2: 256 rows (q, nb) of 8, stride 9
  static constexpr int LDS = B2 + 256 * 9;   // complex elements
};
template <>
struct Shape<4096> {
  static constexpr int NT = 256;
  static constexpr int TW2 = 16;             // w256^(q c)
  static constexpr int RS1 = 272;            // both buffers: 16 rows of 256, padded
  static constexpr int B2 = 16 * RS1;
  static constexpr int LDS = 32 * RS1;
};
template <>
struct Shape<8192> {
  static constexpr int NT = 512;
  static constexpr int TW2 = 32;             // w512^(q c); row 16 holds w32^p, p < 16
  static constexpr int RS1 = 512;            // buffer 1: 16 rows of 512 (also buffer 3)
  static constexpr int B2 = 16 * RS1;        // buffer 2: 256 rows (q, nb) of 32, stride 33
  static constexpr int LDS = B2 + 256 * 33;
};

// C-point DFT with exponent sign S over the workgroup.
// In:  v[r] = x[tid + NT r].  Out: v[r] = X[tid + NT r].
// tw1[nb-1] = w_C^(nb*tid), tw2[q-1] = w_M^(q*(tid mod TW2)) (positive
// exponents, M = C/16); tw3[p] = w32^p (C = 8192 only).
template <int C, int S>
__device__ __forceinline__ void fft_chunk(float2 (&v)[16], const float2 (&tw1)[15], const float2 (&tw2)[15],
                                          const float2* __restrict__ tw3, float2* __restrict__ lds, int tid) {
  using Sh = Shape<C>;
  // pass 1: over r, then twiddle by w_C^(nb*t); element (nb, t) -> buffer 1 row nb
  fft16<S>(v);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int nb = perm16(p);
    float2 a = v[p];
    if (nb != 0) a = ctw<S>(a, tw1[nb - 1]);
    lds[nb * Sh::RS1 + tid] = a;
  }
  __syncthreads();
  if constexpr (C == 4096) {
    float2* buf2 = lds + Sh::B2;
    // pass 2: thread (nb2, c), transform over d of element (nb2, c + 16 d)
    {
      const int nb2 = tid >> 4, c = tid & 15;
#pragma unroll
      for (int d = 0; d < 16; ++d) v[d] = lds[nb2 * Sh::RS1 + c + 16 * d];
      fft16<S>(v);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int q = perm16(p);
        float2 a = v[p];
        if (q != 0) a = ctw<S>(a, tw2[q - 1]);
        buf2[q * Sh::RS1 + 16 * nb2 + (c ^ nb2)] = a;
      }
    }
    __syncthreads();
    // pass 3: thread (q3, nb3), transform over c
    {
      const int q3 = tid >> 4, nb3 = tid & 15;
#pragma unroll
      for (int c = 0; c < 16; ++c) v[c] = buf2[q3 * Sh::RS1 + 16 * nb3 + (c ^ nb3)];
      fft16<S>(v);
    }
    // v[p] now holds X[tid + 256 * perm16(p)]; restore natural register order.
    float2 t[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) t[r] = v[perm16(r)];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = t[r];
  } else if constexpr (C == 2048) {
    float2* buf2 = lds + Sh::B2;
    // pass 2: thread (nb2, c), c < 8: transform over d of element (nb2, c + 8 d),
    // twiddle w128^(q c); element (q, nb2, c) -> buf2[(16 q + nb2) * 9 + c]
    {
      const int nb2 = tid >> 3, c = tid & 7;
#pragma unroll
      for (int d = 0; d < 16; ++d) v[d] = lds[nb2 * Sh::RS1 + c + 8 * d];
      fft16<S>(v);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int q = perm16(p);
        float2 a = v[p];
        if (q != 0) a = ctw<S>(a, tw2[q - 1]);
        buf2[(16 * q + nb2) * 9 + c] = a;
      }
    }
    __syncthreads();
    // pass 3: thread (nb3, qlo) transforms over c for q = qlo and qlo + 8;
    // output p of q = qlo + 8 h is X[nb3 + 16 q + 256 p] = X[tid + 128 (h + 2 p)]
    {
      const int nb3 = tid & 15, qlo = tid >> 4;
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int c = 0; c < 8; ++c) v[8 * h + c] = buf2[(16 * (qlo + 8 * h) + nb3) * 9 + c];
      dft8<S>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]);
      dft8<S>(v[8], v[9], v[10], v[11], v[12], v[13], v[14], v[15]);
    }
    float2 t[16];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int p = 0; p < 8; ++p) t[h + 2 * p] = v[8 * h + p];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = t[r];
  } else {
    static_assert(C == 8192, "chunk lengths 2048, 4096, 8192");
    float2* buf2 = lds + Sh::B2;
    // pass 2: thread (nb2, c), c < 32: transform over d of element (nb2, c + 32 d),
    // twiddle w512^(q c); element (q, nb2, c) -> buf2[(16 q + nb2) * 33 + c]
    {
      const int nb2 = tid >> 5, c = tid & 31;
#pragma unroll
      for (int d = 0; d < 16; ++d) v[d] = lds[nb2 * Sh::RS1 + c + 32 * d];
      fft16<S>(v);
#pragma unroll
      for (int p = 0; p < 16; ++p) {
        const int q = perm16(p);
        float2 a = v[p];
        if (q != 0) a = ctw<S>(a, tw2[q - 1]);
        buf2[(16 * q + nb2) * 33 + c] = a;
      }
    }
    __syncthreads();
    // pass 3a: the 32-point DFT over c = c0 + 2 c1 of row l = (q, nb): thread
    // (c0, l), c0 = tid / 256 uniform per wave, transforms over c1 (index p1)
    // and multiplies by w32^(p1 c0); element (p1, c0, l) -> buffer 1
    // [(2 p1 + c0) * 256 + l]
    {
      const int c0 = tid >> 8, l = tid & 255;
#pragma unroll
      for (int c1 = 0; c1 < 16; ++c1) v[c1] = buf2[l * 33 + c0 + 2 * c1];
      fft16<S>(v);
      if (c0) {
#pragma unroll
        for (int p = 0; p < 16; ++p) {
          const int p1 = perm16(p);
          if (p1 != 0) v[p] = ctw<S>(v[p], tw3[p1]);
        }
      }
#pragma unroll
      for (int p = 0; p < 16; ++p) lds[(2 * perm16(p) + c0) * 256 + l] = v[p];
    }
    __syncthreads();
    // pass 3b: radix 2 over c0: output p = p1 + 16 p2 of row l is
    // X[l + 256 p1 + 4096 p2]; thread (p1lo, l) takes p1 = p1lo + 2 m, so
    // register m + 8 p2 holds X[tid + 512 (m + 8 p2)]
    {
      const int p1lo = tid >> 8, l = tid & 255;
#pragma unroll
      for (int m = 0; m < 8; ++m) {
        const int p1 = p1lo + 2 * m;
        const float2 a = lds[(2 * p1) * 256 + l];
        const float2 b = lds[(2 * p1 + 1) * 256 + l];
        v[m] = cadd(a, b);
        v[m + 8] = csub(a, b);
      }
    }
    // the next transform writes buffer 1 again
    __syncthreads();
  }
}

// Buffer resource (gfx9 layout, raw access) over `bytes` bytes at `base`.
// Stores at byte offsets >= bytes are dropped by the hardware range check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// Twiddles of one chunk length, as each thread uses them.
struct Tw {
  float2 tw1[15];
  float2 tw2[15];
  const float2* tw3;
};

// One template: v = F * H_z, inverse FFT, |y|^2 of the valid outputs.
// hc holds H_z (this thread's 16 bins); hn receives H_{z+1} when next_ok.
template <int C>
__device__ __forceinline__ void ols_template(const float2 (&F)[16], const float2 (&hc)[16], float2 (&hn)[16],
                                             bool next_ok, const float2* __restrict__ Hnext,
                                             float* __restrict__ out_row, uint32_t out_bytes, const Tw& tw,
                                             float2* __restrict__ lds, int tid) {
  constexpr int NT = Shape<C>::NT;
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = cmul(F[r], hc[r]);
  if (next_ok) {
#pragma unroll
    for (int r = 0; r < 16; ++r) hn[r] = Hnext[tid + NT * r];
  }
  fft_chunk<C, 1>(v, tw.tw1, tw.tw2, tw.tw3, lds, tid);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(out_row, out_bytes);
  // Non-temporal stores (cache policy NT = 2): the FOP is written once here and
  // next read by the harmonic sum after the whole plane is done, so keeping it
  // in L2 / the memory-side cache only leaves dirty lines whose write-back
  // competes with that kernel's reads (measured: harmonic sum 0.42 -> 0.35 ms
  // after the convolution of a 2^22-bin spectrum).
#pragma unroll
  for (int r = 0; r < 16; ++r)
    // the b32 store takes raw bits: pass the float's bit pattern, not a converted value
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v[r].x * v[r].x + v[r].y * v[r].y), rs,
                                          (int)((tid + NT * r) * 4), 0, 2);
}

// The zero-drift template is a unit delta (its response A(q, 0) vanishes at
// every non-zero integer q), so its row is |X|^2 of the chunk's valid bins:
// written from the input directly, with no transform.
template <int C>
__device__ __forceinline__ void delta_row(const float2* __restrict__ x, int64_t base, float* __restrict__ out_row,
                                          uint32_t out_bytes, int tid) {
  constexpr int NT = Shape<C>::NT;
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(out_row, out_bytes);
  const int lim = (int)(out_bytes / 4u);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int s = tid + NT * r;
    float p = 0.0f;
    if (s < lim) {
      const float2 a = x[base + s];
      p = a.x * a.x + a.y * a.y;
    }
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(p), rs, s * 4, 0, 2);
  }
}

// One work item: chunk `chunk` of spectrum x (n bins) and templates
// [z_lo, z_hi): forward FFT once, then per template multiply, inverse FFT and
// power of the valid outputs into fop (row stride ld).  Row zrow (the
// zero-drift template) is |X|^2 and is written without a transform.
template <int C>
__device__ __forceinline__ void ols_item(const float2* __restrict__ x, int64_t n, float* __restrict__ fop,
                                         int64_t ld, const float2* __restrict__ H, int64_t chunk, int z_lo,
                                         int z_hi, int zrow, int V, int P, const Tw& tw, float2* __restrict__ lds,
                                         int tid) {
  constexpr int NT = Shape<C>::NT;
  const int64_t base = chunk * V;
  // valid outputs of this chunk: s < V and base + s < n
  const int64_t lim64 = n - base < (int64_t)V ? n - base : (int64_t)V;
  const uint32_t out_bytes = (uint32_t)lim64 * 4u;
  // templates to transform: [z_lo, z_hi) without the delta row, as the two
  // segments [z_lo, skip) and [skip + 1, z_hi) (uniform)
  const bool has_delta = zrow >= z_lo && zrow < z_hi;
  if (has_delta) {
    delta_row<C>(x, base, fop + (size_t)zrow * ld + base, out_bytes, tid);
    if (z_hi - z_lo == 1) return;
  }
  const int skip = has_delta ? zrow : z_hi;
  float2 v[16];
  const int64_t in0 = base - P + tid;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t idx = in0 + NT * r;
    v[r] = (idx >= 0 && idx < n) ? x[idx] : make_float2(0.0f, 0.0f);
  }
  fft_chunk<C, -1>(v, tw.tw1, tw.tw2, tw.tw3, lds, tid);
  float2 F[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) F[r] = v[r];

  float2 hA[16], hB[16];
  for (int seg = 0; seg < 2; ++seg) {
    const int s0 = seg == 0 ? z_lo : skip + 1, s1 = seg == 0 ? skip : z_hi;
    if (s0 >= s1) continue;  // uniform
    {
      const float2* Hz = H + (size_t)s0 * C;
#pragma unroll
      for (int r = 0; r < 16; ++r) hA[r] = Hz[tid + NT * r];
    }
    // two templates per trip with ping-pong prefetch buffers (no register copies)
    for (int z = s0; z < s1; z += 2) {
      ols_template<C>(F, hA, hB, z + 1 < s1, H + (size_t)(z + 1) * C, fop + (size_t)z * ld + base, out_bytes, tw,
                      lds, tid);
      if (z + 1 < s1)
        ols_template<C>(F, hB, hA, z + 2 < s1, H + (size_t)(z + 2) * C, fop + (size_t)(z + 1) * ld + base,
                        out_bytes, tw, lds, tid);
    }
  }
}

// tw1tab[k][t] = w_C^(k t) (t < NT), tw2tab[k][c] = w_M^(k c) (c < TW2), row 16
// of tw2tab = w32^p (C = 8192)
template <int C>
__device__ __forceinline__ void load_twiddles(const float2* __restrict__ tw1tab, const float2* __restrict__ tw2tab,
                                              Tw& tw, int tid) {
  constexpr int NT = Shape<C>::NT, TW2 = Shape<C>::TW2;
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    tw.tw1[k - 1] = tw1tab[k * NT + tid];
    tw.tw2[k - 1] = tw2tab[k * TW2 + (tid & (TW2 - 1))];
  }
  tw.tw3 = tw2tab + 16 * TW2;
}

// Work split of the persistent grid.  The (chunk, template) pairs, chunk-major
// (pair q = chunk * rows + z), are cut into gridDim.x contiguous ranges of
// equal length; a workgroup transforms a chunk forward once for every chunk its
// range touches (at most tmax templates per forward transform).  Every
// workgroup does the same number of inverse transforms plus two or three
// forward ones, so the grid finishes together.
__device__ __forceinline__ void pair_range(int64_t total, int64_t& lo, int64_t& hi) {
  lo = total * (int64_t)blockIdx.x / (int64_t)gridDim.x;
  hi = total * ((int64_t)blockIdx.x + 1) / (int64_t)gridDim.x;
}

// templates [z_lo, z_hi) of the piece of the range [q, hi) that starts at pair q
__device__ __forceinline__ int piece_end(int64_t q, int64_t hi, int z_lo, int rows, int tmax) {
  return (int)min((int64_t)min(rows, z_lo + tmax), (int64_t)z_lo + (hi - q));
}

template <int C>
__global__ __launch_bounds__(Shape<C>::NT, 2) void k_ols_conv(const float2* __restrict__ x, int64_t n,
                                                              float* __restrict__ fop, int64_t ld,
                                                              const float2* __restrict__ H,
                                                              const float2* __restrict__ tw1tab,
                                                              const float2* __restrict__ tw2tab, int rows, int tmax,
                                                              int64_t chunks, int V, int P) {
  __shared__ float2 lds[Shape<C>::LDS];
  const int tid = threadIdx.x;
  Tw tw;
  load_twiddles<C>(tw1tab, tw2tab, tw, tid);
  int64_t q, hi;
  pair_range(chunks * rows, q, hi);
  while (q < hi) {
    const int64_t chunk = q / rows;
    const int z_lo = (int)(q - chunk * rows);
    const int z_hi = piece_end(q, hi, z_lo, rows, tmax);
    ols_item<C>(x, n, fop, ld, H, chunk, z_lo, z_hi, rows / 2, V, P, tw, lds, tid);
    q += z_hi - z_lo;
  }
}

// Listed chunks only, templates z0 .. z0 + nr - 1: pair q = i * nr + (z - z0)
// over chunk_list[0 .. nlist); with d_nlist the list length is read from
// device memory (written by an earlier kernel on the stream).
template <int C>
__global__ __launch_bounds__(Shape<C>::NT, 2) void k_ols_conv_list(const float2* __restrict__ x, int64_t n,
                                                                   float* __restrict__ fop, int64_t ld,
                                                                   const float2* __restrict__ H,
                                                                   const float2* __restrict__ tw1tab,
                                                                   const float2* __restrict__ tw2tab, int z0, int nr,
                                                                   const int* __restrict__ chunk_list, int nlist,
                                                                   const int* __restrict__ d_nlist, int zrow, int V,
                                                                   int P) {
  __shared__ float2 lds[Shape<C>::LDS];
  const int tid = threadIdx.x;
  if (d_nlist) nlist = *d_nlist;
  Tw tw;
  load_twiddles<C>(tw1tab, tw2tab, tw, tid);
  int64_t q, hi;
  pair_range((int64_t)nlist * nr, q, hi);
  while (q < hi) {
    const int64_t li = q / nr;
    const int r_lo = (int)(q - li * nr);
    const int r_hi = piece_end(q, hi, r_lo, nr, nr);
    ols_item<C>(x, n, fop, ld, H, chunk_list[li], z0 + r_lo, z0 + r_hi, zrow, V, P, tw, lds, tid);
    q += r_hi - r_lo;
  }
}

// Batch of spectra: trial t owns pairs [trials[t].item0, trials[t+1].item0)
// (its chunks x rows); this launch splits pairs [item_begin, item_end).  A
// piece never crosses a chunk, hence never a trial.
template <int C>
__global__ __launch_bounds__(Shape<C>::NT, 2) void k_ols_conv_batch(const ConvTrial* __restrict__ trials, int ntrials,
                                                                    int64_t item_begin, int64_t item_end,
                                                                    const float2* __restrict__ H,
                                                                    const float2* __restrict__ tw1tab,
                                                                    const float2* __restrict__ tw2tab, int rows,
                                                                    int tmax, int V, int P) {
  __shared__ float2 lds[Shape<C>::LDS];
  const int tid = threadIdx.x;
  Tw tw;
  load_twiddles<C>(tw1tab, tw2tab, tw, tid);
  int64_t q, hi;
  pair_range(item_end - item_begin, q, hi);
  q += item_begin;
  hi += item_begin;
  while (q < hi) {
    // last trial whose first pair is <= q (uniform across the workgroup)
    int lo = 0, up = ntrials - 1;
    while (lo < up) {
      const int mid = (lo + up + 1) >> 1;
      if (trials[mid].item0 <= q) lo = mid; else up = mid - 1;
    }
    const ConvTrial tr = trials[lo];
    const int64_t local = q - tr.item0;
    const int64_t chunk = local / rows;
    const int z_lo = (int)(local - chunk * rows);
    const int z_hi = piece_end(q, hi, z_lo, rows, tmax);
    ols_item<C>(tr.x, tr.n, tr.fop, tr.ld, H, chunk, z_lo, z_hi, rows / 2, V, P, tw, lds, tid);
    q += z_hi - z_lo;
  }
}

}  // namespace

int ols_threads(int C) { return C / 16; }

bool ols_chunk_built(int C) { return C == 2048 || C == 4096 || C == 8192; }

int ols_slots_per_cu(int C) {
  // resident workgroups per compute unit at two waves per SIMD (LDS allowing)
  return C == 2048 ? 4 : (C == 4096 ? 2 : 1);
}

hipError_t launch_ols_conv(const float2* x, int64_t n, float* fop, int64_t ld, const OlsTables& t, int rows,
                           int slots, hipStream_t s) {
  const OlsGeom& g = t.geom;
  const int64_t chunks = (n + g.V - 1) / g.V;
  const unsigned grid = (unsigned)std::min<int64_t>(chunks * rows, slots);
  switch (g.C) {
#define FDAS_OLS_CASE(CC)                                                                                          \
  case CC:                                                                                                         \
    hipLaunchKernelGGL(k_ols_conv<CC>, dim3(grid), dim3(Shape<CC>::NT), 0, s, x, n, fop, ld, t.H, t.tw1, t.tw2,    \
                       rows, rows, chunks, g.V, g.P);                                                              \
    break;
    FDAS_OLS_CASE(2048)
    FDAS_OLS_CASE(4096)
    FDAS_OLS_CASE(8192)
#undef FDAS_OLS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ols_conv_list(const float2* x, int64_t n, float* fop, int64_t ld, const OlsTables& t, int z0,
                                int nr, int zrow, int slots, const int* chunk_list, int nlist, hipStream_t s,
                                const int* d_nlist) {
  if (nlist <= 0 || nr <= 0) return hipSuccess;
  const OlsGeom& g = t.geom;
  const unsigned grid = (unsigned)std::min<int64_t>((int64_t)nlist * nr, slots);
  switch (g.C) {
#define FDAS_OLS_CASE(CC)                                                                                          \
  case CC:                                                                                                         \
    hipLaunchKernelGGL(k_ols_conv_list<CC>, dim3(grid), dim3(Shape<CC>::NT), 0, s, x, n, fop, ld, t.H, t.tw1,      \
                       t.tw2, z0, nr, chunk_list, nlist, d_nlist, zrow, g.V, g.P);                                 \
    break;
    FDAS_OLS_CASE(2048)
    FDAS_OLS_CASE(4096)
    FDAS_OLS_CASE(8192)
#undef FDAS_OLS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_ols_conv_batch(const ConvTrial* trials, int ntrials, int64_t item_begin, int64_t item_end,
                                 const OlsTables& t, int rows, int tmax, int slots, hipStream_t s) {
  if (item_end <= item_begin) return hipSuccess;
  const OlsGeom& g = t.geom;
  const unsigned grid = (unsigned)std::min<int64_t>(item_end - item_begin, slots);
  const int tm = tmax > 0 ? std::min(tmax, rows) : rows;
  switch (g.C) {
#define FDAS_OLS_CASE(CC)                                                                                          \
  case CC:                                                                                                         \
    hipLaunchKernelGGL(k_ols_conv_batch<CC>, dim3(grid), dim3(Shape<CC>::NT), 0, s, trials, ntrials, item_begin,   \
                       item_end, t.H, t.tw1, t.tw2, rows, tm, g.V, g.P);                                           \
    break;
    FDAS_OLS_CASE(2048)
    FDAS_OLS_CASE(4096)
    FDAS_OLS_CASE(8192)
#undef FDAS_OLS_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace fdas
