// Overlap-save FFT correlation of a complex spectrum with every acceleration
// template, fused with the power and the discard of the overlap
// (Section 2.1.2 overlap-save FDFIR, eq. (2); power as in Section 2.2).
//
// One workgroup = one chunk of C = 4096 input bins and a group of templates.
//   chunk c covers outputs j in [c*V, c*V + V), V = C - (L_max - 1), and reads
//   X[c*V - P + t], t in [0, C), P = L_max/2, zero outside [0, n).
//   F = FFT(chunk) once (shared by all templates of the group, as the
//   area-efficient AOLS design of Section 2.1.3 transforms the input once),
//   then per template: y = IFFT(F * H_z), |y|^2 of the first V outputs -> FOP.
//   H_z = (1/C) * sum_t g_z[t] e^{+2 pi i t k / C} with g_z the template placed
//   at t = P + d, so y[s] = sum_d X[c*V + s + d] h_z[d] (centred correlation).
//
// The 4096-point FFT runs in three radix-16 passes, 256 threads x 16 points:
//   pass 1: thread t transforms x[t + 256 r] over r (16 points in registers),
//           twiddle w4096^(nb*t), write to LDS buffer 1;
//   pass 2: thread (nb, c) transforms the 16 values c + 16 d over d,
//           twiddle w256^(q*c), write to LDS buffer 2;
//   pass 3: thread (q, nb) transforms over c and ends holding output
//           y[t + 256 p] in register p -- the same layout as the input, so
//           the forward result F stays in registers for every template.
// LDS strides (272 complex per row) and the XOR swizzle of buffer 2 make every
// LDS access of a half-wave hit distinct banks.  No packed-FP32 instructions
// are written here (the build disables them).

#include <algorithm>

#include "fdas_internal.h"
#include "fft16.h"

namespace fdas {
namespace {

constexpr int NT = kOlsThreads;   // 256
constexpr int RS = 272;           // LDS row stride, complex elements

using namespace fft;


// 4096-point DFT with exponent sign S over the workgroup.
// In:  v[r] = x[tid + 256 r].  Out: v[r] = X[tid + 256 r].
// tw1[nb-1] = w4096^(nb*tid), tw2[q-1] = w256^(q*(tid & 15)) (positive exponent).
template <int S>
__device__ __forceinline__ void fft4096(float2 (&v)[16], const float2 (&tw1)[15], const float2 (&tw2)[15],
                                        float2* __restrict__ buf1, float2* __restrict__ buf2, int tid) {
  // pass 1: over r, then twiddle by w4096^(nb*t); element (nb, t) -> buf1[nb*RS + t]
  fft16<S>(v);
#pragma unroll
  for (int p = 0; p < 16; ++p) {
    const int nb = perm16(p);
    float2 a = v[p];
    if (nb != 0) a = ctw<S>(a, tw1[nb - 1]);
    buf1[nb * RS + tid] = a;
  }
  __syncthreads();
  // pass 2: thread (nb2, c), transform over d of element (nb2, c + 16 d)
  {
    const int nb2 = tid >> 4, c = tid & 15;
#pragma unroll
    for (int d = 0; d < 16; ++d) v[d] = buf1[nb2 * RS + c + 16 * d];
    fft16<S>(v);
#pragma unroll
    for (int p = 0; p < 16; ++p) {
      const int q = perm16(p);
      float2 a = v[p];
      if (q != 0) a = ctw<S>(a, tw2[q - 1]);
      buf2[q * RS + 16 * nb2 + (c ^ nb2)] = a;
    }
  }
  __syncthreads();
  // pass 3: thread (q3, nb3), transform over c
  {
    const int q3 = tid >> 4, nb3 = tid & 15;
#pragma unroll
    for (int c = 0; c < 16; ++c) v[c] = buf2[q3 * RS + 16 * nb3 + (c ^ nb3)];
    fft16<S>(v);
  }
  // v[p] now holds X[tid + 256 * perm16(p)]; restore natural register order.
  float2 t[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) t[r] = v[perm16(r)];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = t[r];
}

// Buffer resource (gfx9 layout, raw access) over `bytes` bytes at `base`.
// Stores at byte offsets >= bytes are dropped by the hardware range check.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

// One template: v = F * H_z, inverse FFT, |y|^2 of the valid outputs.
// hc holds H_z (this thread's 16 bins); hn receives H_{z+1} when next_ok.
__device__ __forceinline__ void ols_template(const float2 (&F)[16], const float2 (&hc)[16], float2 (&hn)[16],
                                             bool next_ok, const float2* __restrict__ Hnext,
                                             float* __restrict__ out_row, uint32_t out_bytes,
                                             const float2 (&tw1)[15], const float2 (&tw2)[15],
                                             float2* __restrict__ buf1, float2* __restrict__ buf2, int tid) {
  float2 v[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = cmul(F[r], hc[r]);
  if (next_ok) {
#pragma unroll
    for (int r = 0; r < 16; ++r) hn[r] = Hnext[tid + 256 * r];
  }
  fft4096<1>(v, tw1, tw2, buf1, buf2, tid);
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
                                          (int)((tid + 256 * r) * 4), 0, 2);
}

// One work item: chunk `chunk` of spectrum x (n bins) and templates
// [z_lo, z_hi): forward FFT once, then per template multiply, inverse FFT and
// power of the valid outputs into fop (row stride ld).
__device__ __forceinline__ void ols_item(const float2* __restrict__ x, int64_t n, float* __restrict__ fop,
                                         int64_t ld, const float2* __restrict__ H, int64_t chunk, int z_lo,
                                         int z_hi, int V, int P, const float2 (&tw1)[15], const float2 (&tw2)[15],
                                         float2* __restrict__ buf1, float2* __restrict__ buf2, int tid) {
  const int64_t base = chunk * V;
  float2 v[16];
  const int64_t in0 = base - P + tid;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t idx = in0 + 256 * r;
    v[r] = (idx >= 0 && idx < n) ? x[idx] : make_float2(0.0f, 0.0f);
  }
  fft4096<-1>(v, tw1, tw2, buf1, buf2, tid);
  float2 F[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) F[r] = v[r];

  // valid outputs of this chunk: s < V and base + s < n
  const int64_t lim64 = n - base < (int64_t)V ? n - base : (int64_t)V;
  const uint32_t out_bytes = (uint32_t)lim64 * 4u;

  float2 hA[16], hB[16];
  {
    const float2* Hz = H + (size_t)z_lo * kOlsC;
#pragma unroll
    for (int r = 0; r < 16; ++r) hA[r] = Hz[tid + 256 * r];
  }
  // two templates per trip with ping-pong prefetch buffers (no register copies)
  for (int z = z_lo; z < z_hi; z += 2) {
    ols_template(F, hA, hB, z + 1 < z_hi, H + (size_t)(z + 1) * kOlsC, fop + (size_t)z * ld + base, out_bytes,
                 tw1, tw2, buf1, buf2, tid);
    if (z + 1 < z_hi)
      ols_template(F, hB, hA, z + 2 < z_hi, H + (size_t)(z + 2) * kOlsC, fop + (size_t)(z + 1) * ld + base,
                   out_bytes, tw1, tw2, buf1, buf2, tid);
  }
}

__device__ __forceinline__ void load_twiddles(const float2* __restrict__ tw1tab, const float2* __restrict__ tw2tab,
                                              float2 (&tw1)[15], float2 (&tw2)[15], int tid) {
#pragma unroll
  for (int k = 1; k < 16; ++k) {
    tw1[k - 1] = tw1tab[k * 256 + tid];
    tw2[k - 1] = tw2tab[k * 16 + (tid & 15)];
  }
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

__global__ __launch_bounds__(NT, 2) void k_ols_conv(const float2* __restrict__ x, int64_t n,
                                                    float* __restrict__ fop, int64_t ld,
                                                    const float2* __restrict__ H,
                                                    const float2* __restrict__ tw1tab,
                                                    const float2* __restrict__ tw2tab, int rows, int tmax,
                                                    int64_t chunks, int V, int P) {
  __shared__ float2 buf1[16 * RS];
  __shared__ float2 buf2[16 * RS];
  const int tid = threadIdx.x;
  float2 tw1[15], tw2[15];
  load_twiddles(tw1tab, tw2tab, tw1, tw2, tid);
  int64_t q, hi;
  pair_range(chunks * rows, q, hi);
  while (q < hi) {
    const int64_t chunk = q / rows;
    const int z_lo = (int)(q - chunk * rows);
    const int z_hi = piece_end(q, hi, z_lo, rows, tmax);
    ols_item(x, n, fop, ld, H, chunk, z_lo, z_hi, V, P, tw1, tw2, buf1, buf2, tid);
    q += z_hi - z_lo;
  }
}

// Listed chunks only, templates z0 .. z0 + nr - 1: pair q = i * nr + (z - z0)
// over chunk_list[0 .. nlist); with d_nlist the list length is read from
// device memory (written by an earlier kernel on the stream).
__global__ __launch_bounds__(NT, 2) void k_ols_conv_list(const float2* __restrict__ x, int64_t n,
                                                         float* __restrict__ fop, int64_t ld,
                                                         const float2* __restrict__ H,
                                                         const float2* __restrict__ tw1tab,
                                                         const float2* __restrict__ tw2tab, int z0, int nr,
                                                         const int* __restrict__ chunk_list, int nlist,
                                                         const int* __restrict__ d_nlist, int V, int P) {
  __shared__ float2 buf1[16 * RS];
  __shared__ float2 buf2[16 * RS];
  const int tid = threadIdx.x;
  if (d_nlist) nlist = *d_nlist;
  float2 tw1[15], tw2[15];
  load_twiddles(tw1tab, tw2tab, tw1, tw2, tid);
  int64_t q, hi;
  pair_range((int64_t)nlist * nr, q, hi);
  while (q < hi) {
    const int64_t li = q / nr;
    const int r_lo = (int)(q - li * nr);
    const int r_hi = piece_end(q, hi, r_lo, nr, nr);
    ols_item(x, n, fop, ld, H, chunk_list[li], z0 + r_lo, z0 + r_hi, V, P, tw1, tw2, buf1, buf2, tid);
    q += r_hi - r_lo;
  }
}

// Batch of spectra: trial t owns pairs [trials[t].item0, trials[t+1].item0)
// (its chunks x rows); this launch splits pairs [item_begin, item_end).  A
// piece never crosses a chunk, hence never a trial.
__global__ __launch_bounds__(NT, 2) void k_ols_conv_batch(const ConvTrial* __restrict__ trials, int ntrials,
                                                          int64_t item_begin, int64_t item_end,
                                                          const float2* __restrict__ H,
                                                          const float2* __restrict__ tw1tab,
                                                          const float2* __restrict__ tw2tab, int rows, int tmax,
                                                          int V, int P) {
  __shared__ float2 buf1[16 * RS];
  __shared__ float2 buf2[16 * RS];
  const int tid = threadIdx.x;
  float2 tw1[15], tw2[15];
  load_twiddles(tw1tab, tw2tab, tw1, tw2, tid);
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
    ols_item(tr.x, tr.n, tr.fop, tr.ld, H, chunk, z_lo, z_hi, V, P, tw1, tw2, buf1, buf2, tid);
    q += z_hi - z_lo;
  }
}

}  // namespace

hipError_t launch_ols_conv(const float2* x, int64_t n, float* fop, int64_t ld, const float2* H,
                           const float2* tw1, const float2* tw2, int rows, const OlsGeom& g, int slots,
                           hipStream_t s) {
  const int64_t chunks = (n + g.V - 1) / g.V;
  const unsigned grid = (unsigned)std::min<int64_t>(chunks * rows, slots);
  hipLaunchKernelGGL(k_ols_conv, dim3(grid), dim3(NT), 0, s, x, n, fop, ld, H, tw1, tw2, rows, rows, chunks, g.V,
                     g.P);
  return hipGetLastError();
}

hipError_t launch_ols_conv_list(const float2* x, int64_t n, float* fop, int64_t ld, const float2* H,
                                const float2* tw1, const float2* tw2, int z0, int nr, const OlsGeom& g, int slots,
                                const int* chunk_list, int nlist, hipStream_t s, const int* d_nlist) {
  if (nlist <= 0 || nr <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((int64_t)nlist * nr, slots);
  hipLaunchKernelGGL(k_ols_conv_list, dim3(grid), dim3(NT), 0, s, x, n, fop, ld, H, tw1, tw2, z0, nr, chunk_list,
                     nlist, d_nlist, g.V, g.P);
  return hipGetLastError();
}

hipError_t launch_ols_conv_batch(const ConvTrial* trials, int ntrials, int64_t item_begin, int64_t item_end,
                                 const float2* H, const float2* tw1, const float2* tw2, int rows, int tmax,
                                 const OlsGeom& g, int slots, hipStream_t s) {
  if (item_end <= item_begin) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>(item_end - item_begin, slots);
  hipLaunchKernelGGL(k_ols_conv_batch, dim3(grid), dim3(NT), 0, s, trials, ntrials, item_begin, item_end, H, tw1,
                     tw2, rows, tmax > 0 ? std::min(tmax, rows) : rows, g.V, g.P);
  return hipGetLastError();
}

}  // namespace fdas
