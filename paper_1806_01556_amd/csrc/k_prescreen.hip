// Learned block pre-screen: a 1D convolutional network over the zero-drift
// power of 4096-bin blocks (not part of the paper's method; a screen that
// decides which blocks need the full search).  Training and inference
// kernels, BF16 weights with FP32 accumulation and FP32 activations.
//
//   a0[t] = log(1 + |X[t]|^2), t < 4096
//   a_l = maxpool4(relu(conv(a_{l-1}; W_l, b_l))), l = 1..3  (1->32->32->32 channels)
//   h   = max_t relu(conv(a_3; W_4, b_4))                     (32 channels)
//   logit = wf . h + bf
//   conv(x; W, b)[o][t] = b[o] + sum_i sum_{k<9} W[o][i][k] x[i][t + k - 4]  (zero outside)
//   loss = w y softplus(-logit) + (1 - y) softplus(logit)   (mean over the batch)
//
// A conv thread owns 32 consecutive outputs of one channel and walks the
// input channels with the 9 weights and a 40-value window of the input in
// registers (288 FMAs per 49 LDS reads).  The data gradient of a layer is the
// same loop with the kernel transposed and flipped; its epilogue routes each
// gradient through the lower layer's max-pool and ReLU.  Weight gradients are
// summed over a tile of positions and a group of samples in registers before
// one atomic add per weight and workgroup.

#include "fdas_internal.h"

namespace fdas {
namespace {

constexpr int PC = 32;      // channels
constexpr int PK = 9;       // kernel taps
constexpr int PT = 256;     // conv outputs per workgroup tile
constexpr int PQ = 32;      // conv outputs per thread
constexpr int PBLK = 4096;  // bins per block

__device__ __forceinline__ float bf16_to_f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ unsigned short f_to_bf16(float v) {
  const __bf16 h = (__bf16)v;  // round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}

__device__ __forceinline__ float softplus(float x) { return log1pf(expf(-fabsf(x))) + fmaxf(x, 0.0f); }

// features of listed blocks: out[b][t] = log(1 + |X[4096 blocks[b] + t]|^2), 0 past n
__global__ void k_ps_features(const float2* __restrict__ x, int64_t n, const int* __restrict__ blocks, int nb,
                              float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nb * PBLK) return;
  const int b = (int)(i / PBLK), t = (int)(i % PBLK);
  const int64_t j = (int64_t)(blocks ? blocks[b] : b) * PBLK + t;  // no list: blocks 0 .. nb-1
  float v = 0.0f;
  if (j < n) {
    const float2 c = x[j];
    v = log1pf(c.x * c.x + c.y * c.y);
  }
  out[i] = v;
}

// One conv tile: x [CIN][L] of sample blockIdx.y, outputs [PT) of tile blockIdx.x.
// mode 0: forward, relu + maxpool4 -> out [PC][L/4] (+ arg), or relu only if pool == 1;
// mode 1: data gradient, w holds the transposed flipped kernel, no bias; the
//         result dx[i][p] is routed into dz_below[i][4p + arg[i][p]] when
//         act[i][p] > 0 (dense, zeros elsewhere).
template <int CIN, int MODE>
__global__ __launch_bounds__(256) void k_ps_conv(const float* __restrict__ x, int L, const unsigned short* __restrict__ w,
                                                 const unsigned short* __restrict__ bias, int pool,
                                                 float* __restrict__ out, unsigned char* __restrict__ arg,
                                                 const float* __restrict__ act_below,
                                                 const unsigned char* __restrict__ arg_below) {
  // row u of the tile at word u + u / 32: the 8 threads of a channel read
  // windows 32 positions apart, which then fall in different banks
  constexpr int XW = PT + 8 + (PT + 8) / 32 + 1;
  __shared__ float xs[CIN][XW];
  __shared__ unsigned short ws[PC][CIN][PK];
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * PT;
  const int tid = threadIdx.x;
  const float* xb = x + (size_t)b * CIN * L;
  for (int e = tid; e < CIN * (PT + 8); e += 256) {
    const int i = e / (PT + 8), u = e % (PT + 8);
    const int t = t0 + u - 4;
    xs[i][u + u / 32] = (t >= 0 && t < L) ? xb[(size_t)i * L + t] : 0.0f;
  }
  for (int e = tid; e < PC * CIN * PK; e += 256) (&ws[0][0][0])[e] = w[e];
  __syncthreads();
  const int o = tid / 8, sub = tid % 8;
  const int q0 = sub * PQ;  // first output of this thread inside the tile
  if (t0 + q0 >= L) return;
  float acc[PQ];
  const float bo = MODE == 0 ? bf16_to_f(bias[o]) : 0.0f;
#pragma unroll
  for (int q = 0; q < PQ; ++q) acc[q] = bo;
  for (int i = 0; i < CIN; ++i) {
    float wk[PK], xw[PQ + 8];
#pragma unroll
    for (int k = 0; k < PK; ++k) wk[k] = bf16_to_f(ws[o][i][k]);
#pragma unroll
    for (int u = 0; u < PQ + 8; ++u) xw[u] = xs[i][q0 + u + (q0 + u) / 32];
#pragma unroll
    for (int q = 0; q < PQ; ++q)
#pragma unroll
      for (int k = 0; k < PK; ++k) acc[q] = fmaf(wk[k], xw[q + k], acc[q]);
  }
  if (MODE == 0) {
    if (pool == 4) {
      // the thread's 8 pooled values are consecutive (32-byte aligned: t0 + q0
      // is a multiple of 32 and Lp of 8): two 16-byte stores, and the max-pool
      // positions as one 8-byte store (training only)
      const int Lp = L / 4;
      float best[PQ / 4];
      unsigned char ba[PQ / 4];
#pragma unroll
      for (int p = 0; p < PQ / 4; ++p) {
        best[p] = fmaxf(acc[4 * p], 0.0f);
        ba[p] = 0;
#pragma unroll
        for (int qq = 1; qq < 4; ++qq) {
          const float v = fmaxf(acc[4 * p + qq], 0.0f);
          if (v > best[p]) {
            best[p] = v;
            ba[p] = (unsigned char)qq;
          }
        }
      }
      static_assert(PQ / 4 == 8, "8 pooled values per thread");
      const size_t o0 = ((size_t)b * PC + o) * Lp + (t0 + q0) / 4;
      float4* dst = reinterpret_cast<float4*>(out + o0);
      dst[0] = make_float4(best[0], best[1], best[2], best[3]);
      dst[1] = make_float4(best[4], best[5], best[6], best[7]);
      if (arg) *reinterpret_cast<uint2*>(arg + o0) = *reinterpret_cast<const uint2*>(ba);
    } else {
#pragma unroll
      for (int q = 0; q < PQ; ++q) out[((size_t)b * PC + o) * L + t0 + q0 + q] = fmaxf(acc[q], 0.0f);
    }
  } else {
    // dx[o][t] for the layer below (o indexes its channels here); dense dz below
    const int Lb = L * 4;
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int p = t0 + q0 + q;
      const size_t ia = ((size_t)b * PC + o) * L + p;
      const int a = arg_below[ia];
      const bool on = act_below[ia] > 0.0f;
      float* dz = out + ((size_t)b * PC + o) * Lb + 4 * p;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) dz[qq] = (on && qq == a) ? acc[q] : 0.0f;
    }
  }
}

// Inference form of a 32 -> 32 channel layer on the matrix cores
// (v_mfma_f32_16x16x32_bf16): out[o][t] = sum over kappa = 32 k + i of
// W[o][i][k] x[i][t + k - 4], as a GEMM with M = 32 channels (two 16-row
// tiles), K = 288 taps x channels (9 steps of 32 channels) and N = positions.
// The weights are BF16 already; each activation is carried as hi + lo BF16
// halves, so two products per step keep FP32-level accuracy.  The input tile
// sits in LDS position-major ([position][channel], hi and lo), so a lane's 8
// consecutive channels of one position are one 16-byte read.
typedef float v4fp __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(256) void k_ps_conv_mfma(const float* __restrict__ x, int L,
                                                      const unsigned short* __restrict__ w,
                                                      const unsigned short* __restrict__ bias, int pool,
                                                      float* __restrict__ out) {
  __shared__ uint4 xhi[(PT + 8) * PC / 8];  // [PT + 8][32] bf16
  __shared__ uint4 xlo[(PT + 8) * PC / 8];
  __shared__ unsigned short ws[PC * PC * PK];  // the layer's weights, [o][i][k]
  const int b = blockIdx.y;
  const int t0 = blockIdx.x * PT;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const float* xb = x + (size_t)b * PC * L;
  // weights: coalesced 16-byte copies (PC * PC * PK shorts = 1152 uint4)
  for (int e = tid; e < PC * PC * PK / 8; e += 256)
    reinterpret_cast<uint4*>(ws)[e] = reinterpret_cast<const uint4*>(w)[e];
  // input tile, position-major: thread (u, c) converts channels 8c .. 8c+7 at
  // one position and writes one 16-byte word of each of xhi / xlo (consecutive
  // threads, consecutive words: no bank conflicts)
  for (int e = tid; e < (PT + 8) * 4; e += 256) {
    const int c = e & 3, u = e >> 2;
    const int t = t0 + u - 4;
    unsigned short h8[8], l8[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const float v = (t >= 0 && t < L) ? xb[(size_t)(8 * c + j) * L + t] : 0.0f;
      h8[j] = f_to_bf16(v);
      l8[j] = f_to_bf16(v - bf16_to_f(h8[j]));
    }
    xhi[u * 4 + c] = *reinterpret_cast<const uint4*>(h8);
    xlo[u * 4 + c] = *reinterpret_cast<const uint4*>(l8);
  }
  __syncthreads();
  // A operands: o-tile ot, step k: lane holds W[16 ot + lane%16][8 (lane/16) + e][k], e < 8
  v8bf A[2][PK];
  const int g = lane >> 4, r = lane & 15;
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int k = 0; k < PK; ++k) {
      unsigned short a8[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) a8[e] = ws[((16 * ot + r) * PC + 8 * g + e) * PK + k];
      A[ot][k] = __builtin_bit_cast(v8bf, *reinterpret_cast<uint4*>(a8));
    }
  const int ntile = min(PT, L - t0) / 16;
  for (int tt = wv; tt < ntile; tt += 4) {
    v4fp acc[2] = {v4fp{0.0f, 0.0f, 0.0f, 0.0f}, v4fp{0.0f, 0.0f, 0.0f, 0.0f}};
#pragma unroll
    for (int k = 0; k < PK; ++k) {
      const int u = 16 * tt + r + k;  // LDS row of position t0 + 16 tt + r + k - 4
      const v8bf bh = __builtin_bit_cast(v8bf, xhi[u * (PC / 8) + g]);
      const v8bf bl = __builtin_bit_cast(v8bf, xlo[u * (PC / 8) + g]);
#pragma unroll
      for (int ot = 0; ot < 2; ++ot) {
        acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ot][k], bh, acc[ot], 0, 0, 0);
        acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A[ot][k], bl, acc[ot], 0, 0, 0);
      }
    }
    // lane holds channels o = 16 ot + 4 g + v at position t = t0 + 16 tt + r
    const int t = t0 + 16 * tt + r;
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = 16 * ot + 4 * g + v;
        float y = fmaxf(acc[ot][v] + bf16_to_f(bias[o]), 0.0f);
        if (pool == 4) {
          y = fmaxf(y, __shfl_xor(y, 1));
          y = fmaxf(y, __shfl_xor(y, 2));
          if ((r & 3) == 0) out[((size_t)b * PC + o) * (L / 4) + t / 4] = y;
        } else {
          out[((size_t)b * PC + o) * L + t] = y;
        }
      }
  }
}

// wt[i][o][k] = w[o][i][8 - k]: the data gradient as a forward convolution
__global__ void k_ps_flip(const unsigned short* __restrict__ w, unsigned short* __restrict__ wt, int cin) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= PC * cin * PK) return;
  const int o = e / (cin * PK), i = (e / PK) % cin, k = e % PK;
  wt[((size_t)i * PC + o) * PK + (PK - 1 - k)] = w[e];
}

// Head: h[c] = max_t r4[c][t] (first maximum), logit, loss and dlogit (when
// labels are given); dz4 dense [PC][64] = dlogit wf[c] at (c, t4[c]) if
// r4 > 0; grad of wf, bf (scaled by 1/B).  One wave per sample.
__global__ __launch_bounds__(64) void k_ps_head(const float* __restrict__ r4, const unsigned short* __restrict__ wf,
                                                const unsigned short* __restrict__ bf,
                                                const float* __restrict__ labels, float pos_weight, int nb,
                                                float* __restrict__ logits, float* __restrict__ loss,
                                                float* __restrict__ dz4, float* __restrict__ grad_fc) {
  const int b = blockIdx.x;
  const int c = threadIdx.x;
  __shared__ float hv[PC];
  __shared__ int ht[PC];
  __shared__ float s_dl;
  if (c < PC) {
    const float* r = r4 + ((size_t)b * PC + c) * 64;
    float best = r[0];
    int bt = 0;
    for (int t = 1; t < 64; ++t)
      if (r[t] > best) {
        best = r[t];
        bt = t;
      }
    hv[c] = best;
    ht[c] = bt;
  }
  __syncthreads();
  if (c == 0) {
    float lg = bf16_to_f(bf[0]);
    for (int k = 0; k < PC; ++k) lg = fmaf(bf16_to_f(wf[k]), hv[k], lg);
    logits[b] = lg;
    float dl = 0.0f;
    if (labels) {
      const float y = labels[b];
      const float s = 1.0f / (1.0f + expf(-lg));
      if (loss) atomicAdd(loss, (pos_weight * y * softplus(-lg) + (1.0f - y) * softplus(lg)) / nb);
      dl = (pos_weight * y * (s - 1.0f) + (1.0f - y) * s) / nb;
    }
    s_dl = dl;
  }
  __syncthreads();
  if (!labels || !dz4) return;
  const float dl = s_dl;
  if (c < PC) {
    float* dz = dz4 + ((size_t)b * PC + c) * 64;
    const float* r = r4 + ((size_t)b * PC + c) * 64;
    for (int t = 0; t < 64; ++t) dz[t] = (t == ht[c] && r[t] > 0.0f) ? dl * bf16_to_f(wf[c]) : 0.0f;
    atomicAdd(&grad_fc[c], dl * hv[c]);
  }
  if (c == PC) atomicAdd(&grad_fc[PC], dl);
}

// Weight and bias gradients of one layer: dW[o][i][k] += sum_b sum_t dz[b][o][t] x[b][i][t + k - 4].
// Workgroup = (tile of PT positions, group of SG samples); each thread sums
// its (o, i) pairs in registers, then one atomic per weight.
constexpr int SG = 16;
template <int CIN>
__global__ __launch_bounds__(256) void k_ps_wgrad(const float* __restrict__ dz, const float* __restrict__ x, int L,
                                                  int nb, float* __restrict__ gw, float* __restrict__ gb) {
  __shared__ float xs[CIN][PT + 8];
  __shared__ float ds[PC][PT];
  const int t0 = blockIdx.x * PT;
  const int b0 = blockIdx.y * SG;
  const int tid = threadIdx.x;
  const int T = min(PT, L - t0);
  constexpr int PAIRS = PC * CIN;
  constexpr int PPT = (PAIRS + 255) / 256;
  float acc[PPT][PK];
  float accb = 0.0f;
#pragma unroll
  for (int u = 0; u < PPT; ++u)
#pragma unroll
    for (int k = 0; k < PK; ++k) acc[u][k] = 0.0f;
  for (int b = b0; b < min(nb, b0 + SG); ++b) {
    __syncthreads();
    const float* xb = x + (size_t)b * CIN * L;
    for (int e = tid; e < CIN * (PT + 8); e += 256) {
      const int i = e / (PT + 8), u = e % (PT + 8);
      const int t = t0 + u - 4;
      xs[i][u] = (t >= 0 && t < L) ? xb[(size_t)i * L + t] : 0.0f;
    }
    for (int e = tid; e < PC * PT; e += 256) {
      const int o = e / PT, u = e % PT;
      ds[o][u] = u < T ? dz[((size_t)b * PC + o) * L + t0 + u] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int pr = tid + 256 * u;
      if (pr < PAIRS) {
        const int o = pr / CIN, i = pr % CIN;
        for (int t = 0; t < T; ++t) {
          const float d = ds[o][t];
#pragma unroll
          for (int k = 0; k < PK; ++k) acc[u][k] = fmaf(d, xs[i][t + k], acc[u][k]);
        }
      }
    }
    if (tid < PC)
      for (int t = 0; t < T; ++t) accb += ds[tid][t];
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int pr = tid + 256 * u;
    if (pr < PAIRS) {
      const int o = pr / CIN, i = pr % CIN;
#pragma unroll
      for (int k = 0; k < PK; ++k) atomicAdd(&gw[((size_t)o * CIN + i) * PK + k], acc[u][k]);
    }
  }
  if (tid < PC) atomicAdd(&gb[tid], accb);
}

// Adam on the FP32 master parameters, then the BF16 copy; clears the gradient.
__global__ void k_ps_adam(float* __restrict__ theta, float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, unsigned short* __restrict__ wb, int np, float lr, float b1, float b2,
                          float c1, float c2, float eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float th = theta[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  theta[i] = th;
  wb[i] = f_to_bf16(th);
  g[i] = 0.0f;
}

__global__ void k_ps_round(const float* __restrict__ theta, unsigned short* __restrict__ wb, int np) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) wb[i] = f_to_bf16(theta[i]);
}

__global__ void k_ps_zero(float* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// Device-side block selection of the pre-screened search (one workgroup):
//   flagged blocks b (logit > threshold) and their harmonic closure, the
//   blocks [m b, m (b + 1) - 1] of the multiples m j, m = 2..nh, of their
//   columns (clipped to the spectrum), are searched;
//   the blocks the searched blocks' harmonic sums read as stretched sources
//   (the sources floor(j/k), floor(j/k) + 1 of each 4-column group, k =
//   2..nh) need only the source rows;
//   overlap-save chunks whose valid outputs touch a searched block are
//   convolved for every template, chunks that touch only source blocks for
//   the source rows; the searched blocks' harmonic-sum tiles are listed.
// lists = [searched chunks, cap_c][tiles, cap_t, tail -1][source-only chunks,
//          cap_c][n_searched_chunks, n_tiles, n_source_chunks]
// The same selection as the host side of fdas_search_blocks with the
// closure of the flagged blocks as its list.
constexpr int kSelThreads = 1024;
constexpr int kPsBlock = PBLK;

__device__ __forceinline__ int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

// exclusive prefix of v over the workgroup; *total receives the sum
__device__ __forceinline__ int block_exclusive_scan(int v, int* s_scan, int* total) {
  const int t = threadIdx.x;
  s_scan[t] = v;
  __syncthreads();
  for (int o = 1; o < kSelThreads; o <<= 1) {
    const int u = t >= o ? s_scan[t - o] : 0;
    __syncthreads();
    s_scan[t] += u;
    __syncthreads();
  }
  const int incl = s_scan[t];
  *total = s_scan[kSelThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ __launch_bounds__(kSelThreads) void k_ps_search_lists(const float* __restrict__ logits, float thr,
                                                                 int64_t n, int nblk, int nh, int V, int tcols,
                                                                 int* __restrict__ lists, int cap_c, int cap_t) {
  __shared__ unsigned char s_search[kMaxSelBlocks];
  __shared__ unsigned char s_src[kMaxSelBlocks];
  __shared__ int s_scan[kSelThreads];
  const int t = threadIdx.x;
  for (int b = t; b < nblk; b += kSelThreads) {
    s_search[b] = 0;
    s_src[b] = 0;
  }
  __syncthreads();
  for (int f = t; f < nblk; f += kSelThreads) {
    if (!(logits[f] > thr)) continue;  // NaN never flags
    s_search[f] = 1;
    for (int m = 2; m <= nh; ++m) {
      const int64_t lo = (int64_t)m * f * kPsBlock;
      const int64_t hi = min64(n - 1, (int64_t)m * ((int64_t)(f + 1) * kPsBlock - 1) + m - 1);
      for (int64_t q = lo / kPsBlock; q <= hi / kPsBlock && q < nblk; ++q) s_search[q] = 1;
    }
  }
  __syncthreads();
  for (int b = t; b < nblk; b += kSelThreads) {
    if (!s_search[b]) continue;
    const int64_t j0 = (int64_t)b * kPsBlock, j1 = min64(n, j0 + kPsBlock) - 1;
    for (int k = 2; k <= nh; ++k) {
      const int64_t s0 = (j0 / 4 * 4) / k, s1 = min64(n - 1, ((j1 / 4 * 4 + 3) / k) + 1);
      for (int64_t q = s0 / kPsBlock; q <= s1 / kPsBlock; ++q) s_src[q] = 1;
    }
  }
  __syncthreads();
  // chunks, in order: searched (every template) and source-only
  const int64_t nchunks = (n + V - 1) / V;
  int* sl = lists + cap_c + cap_t;
  int base = 0, sbase = 0;
  for (int64_t c0 = 0; c0 < nchunks; c0 += kSelThreads) {
    const int64_t c = c0 + t;
    int full = 0, src = 0;
    if (c < nchunks) {
      const int64_t a = c * V, z = min64(n, a + V) - 1;
      for (int64_t q = a / kPsBlock; q <= z / kPsBlock; ++q) {
        full |= s_search[q];
        src |= s_src[q];
      }
    }
    const int only_src = src && !full;
    int tot, stot;
    const int pos = block_exclusive_scan(full, s_scan, &tot);
    const int spos = block_exclusive_scan(only_src, s_scan, &stot);
    if (full && base + pos < cap_c) lists[base + pos] = (int)c;
    if (only_src && sbase + spos < cap_c) sl[sbase + spos] = (int)c;
    base += tot;
    sbase += stot;
  }
  const int nc = min(base, cap_c), ns = min(sbase, cap_c);
  // tiles of the searched blocks, in order; the rest of the tile list is -1
  const int per = kPsBlock / tcols;
  const int64_t ntiles = (n + tcols - 1) / tcols;
  int* tl = lists + cap_c;
  base = 0;
  for (int b0 = 0; b0 < nblk; b0 += kSelThreads) {
    const int b = b0 + t;
    int cnt = 0;
    if (b < nblk && s_search[b]) cnt = (int)max64(0, min64(per, ntiles - (int64_t)b * per));
    int tot;
    const int pos = block_exclusive_scan(cnt, s_scan, &tot);
    for (int i = 0; i < cnt; ++i)
      if (base + pos + i < cap_t) tl[base + pos + i] = b * per + i;
    base += tot;
  }
  const int nt = min(base, cap_t);
  for (int i = nt + t; i < cap_t; i += kSelThreads) tl[i] = -1;
  if (t == 0) {
    lists[2 * cap_c + cap_t] = nc;
    lists[2 * cap_c + cap_t + 1] = nt;
    lists[2 * cap_c + cap_t + 2] = ns;
  }
}

}  // namespace

// ---- parameter layout --------------------------------------------------------
int ps_param_count() { return (PC * 1 * PK + PC) + 3 * (PC * PC * PK + PC) + PC + 1; }

static int ps_off_w(int l) {  // layer l = 0..3
  int o = 0;
  for (int j = 0; j < l; ++j) o += PC * (j == 0 ? 1 : PC) * PK + PC;
  return o;
}
static int ps_off_b(int l) { return ps_off_w(l) + PC * (l == 0 ? 1 : PC) * PK; }
static int ps_off_fc() { return ps_off_w(4); }

size_t ps_workspace_bytes(int max_batch) {
  const size_t B = (size_t)max_batch;
  // a1, arg1 (1024); a2, arg2 (256); a3, arg3 (64); r4 (64); dz3/dz2/dz1/dz4 buffers
  const size_t floats = B * PC * (1024 + 256 + 64 + 64) + B * PC * (4096 + 1024 + 256 + 64) + B;
  const size_t bytes8 = B * PC * (1024 + 256 + 64);
  return floats * sizeof(float) + bytes8 + 4 * (size_t)PC * PC * PK * sizeof(unsigned short) + 1024;
}

hipError_t ps_forward_backward(const PsBuffers& pb, const float* feats, int nb, const float* labels, float pos_weight,
                               float* logits, float* loss, hipStream_t s) {
  const unsigned short* w = pb.wbf;
  const dim3 blk(256);
  const bool train = labels != nullptr;
  // forward; inference runs the 32-channel layers on the matrix cores, training
  // on the vector units (it also records the max-pool positions)
  hipLaunchKernelGGL((k_ps_conv<1, 0>), dim3(PBLK / PT, nb), blk, 0, s, feats, PBLK, w + ps_off_w(0),
                     w + ps_off_b(0), 4, pb.a1, train ? pb.arg1 : nullptr, nullptr, nullptr);
  if (train) {
    hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1024 / PT, nb), blk, 0, s, pb.a1, 1024, w + ps_off_w(1),
                       w + ps_off_b(1), 4, pb.a2, pb.arg2, nullptr, nullptr);
    hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1, nb), blk, 0, s, pb.a2, 256, w + ps_off_w(2), w + ps_off_b(2), 4,
                       pb.a3, pb.arg3, nullptr, nullptr);
    hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1, nb), blk, 0, s, pb.a3, 64, w + ps_off_w(3), w + ps_off_b(3), 1,
                       pb.r4, nullptr, nullptr, nullptr);
  } else {
    hipLaunchKernelGGL(k_ps_conv_mfma, dim3(1024 / PT, nb), blk, 0, s, pb.a1, 1024, w + ps_off_w(1), w + ps_off_b(1),
                       4, pb.a2);
    hipLaunchKernelGGL(k_ps_conv_mfma, dim3(1, nb), blk, 0, s, pb.a2, 256, w + ps_off_w(2), w + ps_off_b(2), 4,
                       pb.a3);
    hipLaunchKernelGGL(k_ps_conv_mfma, dim3(1, nb), blk, 0, s, pb.a3, 64, w + ps_off_w(3), w + ps_off_b(3), 1,
                       pb.r4);
  }
  hipLaunchKernelGGL(k_ps_head, dim3(nb), dim3(64), 0, s, pb.r4, w + ps_off_fc(), w + ps_off_fc() + PC, labels,
                     pos_weight, nb, logits, loss, train ? pb.dz4 : nullptr, pb.grad + ps_off_fc());
  if (!train) return hipGetLastError();
  // backward: weight gradients of layer 4, then the data gradient into dz3, ...
  hipLaunchKernelGGL(k_ps_wgrad<PC>, dim3(1, (nb + SG - 1) / SG), blk, 0, s, pb.dz4, pb.a3, 64, nb,
                     pb.grad + ps_off_w(3), pb.grad + ps_off_b(3));
  const float* dz_above = pb.dz4;
  float* dz_below[3] = {pb.dz1, pb.dz2, pb.dz3};
  const float* act[3] = {pb.a1, pb.a2, pb.a3};
  const unsigned char* args[3] = {pb.arg1, pb.arg2, pb.arg3};
  const float* xin[4] = {feats, pb.a1, pb.a2, pb.a3};
  const int Lz[4] = {4096, 1024, 256, 64};
  for (int l = 3; l >= 1; --l) {
    // transposed, flipped W_{l+1} (layer index l here is 0-based for the conv below the gradient)
    hipLaunchKernelGGL(k_ps_flip, dim3((PC * PC * PK + 255) / 256), dim3(256), 0, s, w + ps_off_w(l), pb.wflip, PC);
    const int L = Lz[l];  // length of the pooled activation a_l = input of layer l+1
    hipLaunchKernelGGL((k_ps_conv<PC, 1>), dim3((L + PT - 1) / PT, nb), blk, 0, s, dz_above, L, pb.wflip, nullptr, 0,
                       dz_below[l - 1], nullptr, act[l - 1], args[l - 1]);
    // weight gradients of layer l (input x_{l-1}, output gradient dz_below[l-1] at length 4L)
    if (l - 1 == 0)
      hipLaunchKernelGGL(k_ps_wgrad<1>, dim3(4 * L / PT, (nb + SG - 1) / SG), blk, 0, s, dz_below[0], xin[0], 4 * L,
                         nb, pb.grad + ps_off_w(0), pb.grad + ps_off_b(0));
    else
      hipLaunchKernelGGL(k_ps_wgrad<PC>, dim3(4 * L / PT, (nb + SG - 1) / SG), blk, 0, s, dz_below[l - 1],
                         xin[l - 1], 4 * L, nb, pb.grad + ps_off_w(l - 1), pb.grad + ps_off_b(l - 1));
    dz_above = dz_below[l - 1];
  }
  return hipGetLastError();
}

hipError_t ps_features(const float2* x, int64_t n, const int* blocks, int nb, float* out, hipStream_t s) {
  const int64_t total = (int64_t)nb * PBLK;
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_ps_features, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, x, n, blocks, nb, out);
  return hipGetLastError();
}

hipError_t ps_adam(const PsBuffers& pb, float lr, float b1, float b2, float c1, float c2, float eps, hipStream_t s) {
  const int np = ps_param_count();
  hipLaunchKernelGGL(k_ps_adam, dim3((np + 255) / 256), dim3(256), 0, s, pb.theta, pb.grad, pb.m, pb.v, pb.wbf, np, lr,
                     b1, b2, c1, c2, eps);
  return hipGetLastError();
}

hipError_t ps_round(const PsBuffers& pb, hipStream_t s) {
  const int np = ps_param_count();
  hipLaunchKernelGGL(k_ps_round, dim3((np + 255) / 256), dim3(256), 0, s, pb.theta, pb.wbf, np);
  return hipGetLastError();
}

hipError_t ps_zero(float* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_ps_zero, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t ps_search_lists(const float* logits, float thr, int64_t n, int nblk, int nh, int V, int tcols, int* lists,
                           int cap_c, int cap_t, hipStream_t s) {
  if (nblk < 1 || nblk > kMaxSelBlocks) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ps_search_lists, dim3(1), dim3(kSelThreads), 0, s, logits, thr, n, nblk, nh, V, tcols, lists,
                     cap_c, cap_t);
  return hipGetLastError();
}

}  // namespace fdas
