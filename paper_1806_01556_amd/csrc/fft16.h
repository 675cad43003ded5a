// Register-level complex arithmetic and the 16-point DFT used by the
// overlap-save convolution (host and device, so the butterflies can be
// checked on the CPU against a plain DFT).
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {
namespace fft {

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// multiply by w^s with w the stored (positive-exponent) twiddle: S = +1 -> w, S = -1 -> conj(w)
template <int S>
__host__ __device__ __forceinline__ float2 ctw(float2 a, float2 w) {
  if constexpr (S > 0) return cmul(a, w); else return cmulc(a, w);
}

// 4-point DFT with exponent sign S, in place: (a, b, c, d) -> (X0, X1, X2, X3).
template <int S>
__host__ __device__ __forceinline__ void dft4(float2& a, float2& b, float2& c, float2& d) {
  const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = csub(b, d);
  // S*i*t3
  const float2 it3 = S > 0 ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x);
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, it3);
  d = csub(t1, it3);
}

// Second radix-4 layer of the 16-point DFT for row k0 = 1, 2, 3: the row's
// inputs (a, b, c, d) = (v[4k0], v[4k0+1], v[4k0+2], v[4k0+3]) still lack
// their internal twiddles w16^(S m0 k0), and those are folded into fused
// multiply-adds instead of being applied first:
//   * a factor R2 (w^2 = R2 (1 + S i), w^6 = R2 (-1 + S i)) becomes the
//     multiplier of the FMA that adds the value to its partner;
//   * for k0 = 1 and 3, b +- d = w^k0 (b' +- w^(2 k0) d') (w^3 = w^1 w^2,
//     w^9 = w^3 w^6), and w^k0 is written as C1 (1 + S i tan(pi/8)) or
//     C1 (tan(pi/8) + S i), so it costs two FMAs and a C1 that again folds
//     into the final FMAs.
// 24, 20 and 24 operations per row instead of 28, 24 and 28.
constexpr float kR2 = 0.70710678118654752440f;  // 1/sqrt(2)
constexpr float kC1 = 0.92387953251128675613f;  // cos(pi/8)
constexpr float kT1 = 0.41421356237309504880f;  // tan(pi/8)

// (1 + S i) v and (-1 + S i) v
template <int S>
__host__ __device__ __forceinline__ float2 one_pi(float2 v) { return make_float2(v.x - S * v.y, v.y + S * v.x); }
template <int S>
__host__ __device__ __forceinline__ float2 mone_pi(float2 v) { return make_float2(-v.x - S * v.y, S * v.x - v.y); }

// outputs (a, b, c, d) <- (t0 + k u, t1 + S i k w, t0 - k u, t1 - S i k w)
template <int S>
__host__ __device__ __forceinline__ void finish4(float2& a, float2& b, float2& c, float2& d, float2 t0, float2 t1,
                                                 float2 u, float2 w, float k) {
  a = make_float2(fmaf(k, u.x, t0.x), fmaf(k, u.y, t0.y));
  c = make_float2(fmaf(-k, u.x, t0.x), fmaf(-k, u.y, t0.y));
  b = make_float2(fmaf(-S * k, w.y, t1.x), fmaf(S * k, w.x, t1.y));
  d = make_float2(fmaf(S * k, w.y, t1.x), fmaf(-S * k, w.x, t1.y));
}

// row k0 = 1 (twiddles w^1, w^2, w^3) or k0 = 3 (w^3, w^6, w^9)
template <int S, int K0>
__host__ __device__ __forceinline__ void row_odd(float2& a, float2& b, float2& c, float2& d) {
  // c' = w^(2 K0) c = kR2 p: p = (1 + S i) c for K0 = 1, (-1 + S i) c for K0 = 3
  const float2 p = K0 == 1 ? one_pi<S>(c) : mone_pi<S>(c);
  const float2 t0 = make_float2(fmaf(kR2, p.x, a.x), fmaf(kR2, p.y, a.y));
  const float2 t1 = make_float2(fmaf(-kR2, p.x, a.x), fmaf(-kR2, p.y, a.y));
  // g, h = b +- w^(2 K0) d
  const float2 q = K0 == 1 ? one_pi<S>(d) : mone_pi<S>(d);
  const float2 g = make_float2(fmaf(kR2, q.x, b.x), fmaf(kR2, q.y, b.y));
  const float2 h = make_float2(fmaf(-kR2, q.x, b.x), fmaf(-kR2, q.y, b.y));
  // w^K0 g = kC1 u, w^K0 h = kC1 w
  float2 u, w;
  if constexpr (K0 == 1) {  // 1 + S i tan(pi/8)
    u = make_float2(fmaf(-S * kT1, g.y, g.x), fmaf(S * kT1, g.x, g.y));
    w = make_float2(fmaf(-S * kT1, h.y, h.x), fmaf(S * kT1, h.x, h.y));
  } else {  // tan(pi/8) + S i
    u = make_float2(fmaf(kT1, g.x, -S * g.y), fmaf(kT1, g.y, S * g.x));
    w = make_float2(fmaf(kT1, h.x, -S * h.y), fmaf(kT1, h.y, S * h.x));
  }
  finish4<S>(a, b, c, d, t0, t1, u, w, kC1);
}

// row k0 = 2 (twiddles w^2, w^4, w^6)
template <int S>
__host__ __device__ __forceinline__ void row_two(float2& a, float2& b, float2& c, float2& d) {
  const float2 ic = make_float2(-S * c.y, S * c.x);  // w^4 c = S i c
  const float2 t0 = cadd(a, ic), t1 = csub(a, ic);
  // w^2 b + w^6 d = kR2 ((b - d) + S i (b + d)), w^2 b - w^6 d = kR2 ((b + d) + S i (b - d))
  const float2 m = csub(b, d), n = cadd(b, d);
  const float2 u = make_float2(m.x - S * n.y, m.y + S * n.x);
  const float2 w = make_float2(n.x - S * m.y, n.y + S * m.x);
  finish4<S>(a, b, c, d, t0, t1, u, w, kR2);
}

// 16-point DFT, exponent sign S, in registers.  Afterwards v[p] holds output
// index perm16(p) = (p >> 2) + 4 * (p & 3) (digit reversal, an involution).
template <int S>
__host__ __device__ __forceinline__ void fft16(float2 (&v)[16]) {
#pragma unroll
  for (int m0 = 0; m0 < 4; ++m0) dft4<S>(v[m0], v[4 + m0], v[8 + m0], v[12 + m0]);
  // row k0 holds v[4*k0 + m0]; its internal twiddles w16^(S*m0*k0) are folded
  // into the row's radix-4 step
  dft4<S>(v[0], v[1], v[2], v[3]);
  row_odd<S, 1>(v[4], v[5], v[6], v[7]);
  row_two<S>(v[8], v[9], v[10], v[11]);
  row_odd<S, 3>(v[12], v[13], v[14], v[15]);
}

__host__ __device__ constexpr int perm16(int p) { return (p >> 2) + 4 * (p & 3); }

// 8-point DFT, exponent sign S, in place, natural order in and out: the even
// and odd samples are two 4-point DFTs E, O and X[k] = E[k] + w8^(S k) O[k],
// X[k + 4] = E[k] - w8^(S k) O[k], with w8 = R2 (1 + i), w8^2 = i, w8^3 = R2 (-1 + i).
template <int S>
__host__ __device__ __forceinline__ void dft8(float2& x0, float2& x1, float2& x2, float2& x3, float2& x4,
                                              float2& x5, float2& x6, float2& x7) {
  dft4<S>(x0, x2, x4, x6);  // E[0..3] in x0, x2, x4, x6
  dft4<S>(x1, x3, x5, x7);  // O[0..3] in x1, x3, x5, x7
  const float2 o1 = one_pi<S>(x3), o3 = mone_pi<S>(x7);  // / R2
  const float2 w1 = make_float2(kR2 * o1.x, kR2 * o1.y);
  const float2 w2 = make_float2(-S * x5.y, S * x5.x);
  const float2 w3 = make_float2(kR2 * o3.x, kR2 * o3.y);
  const float2 e0 = x0, e1 = x2, e2 = x4, e3 = x6, w0 = x1;
  x0 = cadd(e0, w0);
  x4 = csub(e0, w0);
  x1 = cadd(e1, w1);
  x5 = csub(e1, w1);
  x2 = cadd(e2, w2);
  x6 = csub(e2, w2);
  x3 = cadd(e3, w3);
  x7 = csub(e3, w3);
}

}  // namespace fft
}  // namespace fdas
