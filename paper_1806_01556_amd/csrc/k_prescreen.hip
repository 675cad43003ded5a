// Learned block pre-screen: a 1D convolutional network over the zero-drift
// power of 4096-bin blocks (not part of the paper's method; a screen that
// decides which blocks need the full search).  Training and inference
// kernels, BF16 weights with FP32 accumulation; training keeps FP32
// activations in global memory, inference (k_ps_infer) keeps them in LDS.
//
//   a0[t] = log(1 + |X[t]|^2), t < 4096
//   a_l = maxpool4(relu(conv(a_{l-1}; W_l, b_l))), l = 1..3  (1->32->32->32 channels)
//   h   = max_t relu(conv(a_3; W_4, b_4))                     (32 channels)
//   logit = wf . h + bf
//   conv(x; W, b)[o][t] = b[o] + sum_i sum_{k<9} W[o][i][k] x[i][t + k - 4]  (zero outside)
//   loss = w y softplus(-logit) + (1 - y) softplus(logit)   (mean over the batch)
//
// Training: a conv thread owns 32 consecutive outputs of one channel and walks the
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

// Inference: the whole network of one sample in one workgroup, every
// activation kept in LDS.  Each layer runs on the matrix cores
// (v_mfma_f32_16x16x32_bf16) as a GEMM with M = 16 positions per tile,
// N = 32 output channels (two 16-column tiles) and K = taps x input channels:
// for the 32 -> 32 channel layers out[t][o] = sum over kappa = 32 k + i of
// x[i][t + k - 4] W[o][i][k], 9 steps of K = 32.  The weights are BF16
// already; each activation is carried as hi + lo BF16 halves, so two products
// per step keep FP32-level accuracy.  Activations sit in LDS position-major
// ([position][channel], hi and lo), so a lane's 8 consecutive channels of one
// position are one 16-byte read.  With positions as the M rows a lane's four
// accumulators are 4 consecutive positions of one channel: the max-pool is
// in-lane.  Layer 0 works in tiles of 64 pooled outputs that go straight into
// the layer-1 tile; layer 1 pools into the whole 256-position a2, layer 2 into
// a3 (64 positions), layer 3 into the per-channel maximum.
typedef float v4fp __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

// B operands (weights) of layers 1..3 in lane order: word ((l - 1) * 2 + ot) * PK + k,
// lane holds W_l[16 ot + lane % 16][8 (lane / 16) + e][k], e < 8
constexpr int kPackWords = 3 * 2 * PK * 64;
static_assert(kPackWords * 8 == kPsPackShorts, "packed weight buffer size");

__global__ void k_ps_pack(const unsigned short* __restrict__ w1, const unsigned short* __restrict__ w2,
                          const unsigned short* __restrict__ w3, uint4* __restrict__ pack) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kPackWords) return;
  const int lane = i % 64, k = (i / 64) % PK, ot = (i / (64 * PK)) % 2, l = i / (64 * PK * 2);
  const unsigned short* w = l == 0 ? w1 : (l == 1 ? w2 : w3);
  unsigned short a8[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) a8[e] = w[((16 * ot + lane % 16) * PC + 8 * (lane / 16) + e) * PK + k];
  pack[i] = *reinterpret_cast<const uint4*>(a8);
}

__device__ __forceinline__ void load_w(const uint4* __restrict__ pack, int l, int lane, v8bf (&W)[2][PK]) {
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int k = 0; k < PK; ++k) W[ot][k] = __builtin_bit_cast(v8bf, pack[(((l - 1) * 2 + ot) * PK + k) * 64 + lane]);
}

// 16 positions (LDS rows row0 + r + k, k < 9) x 32 channels; lane (r, g)
// ends with positions 4 g + v, v < 4, of channel 16 ot + r
__device__ __forceinline__ void mfma_tile(const uint4* xh, const uint4* xl, int row0, const v8bf (&W)[2][PK], int r,
                                          int g, v4fp (&acc)[2]) {
  acc[0] = v4fp{0.0f, 0.0f, 0.0f, 0.0f};
  acc[1] = v4fp{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < PK; ++k) {
    const int u = row0 + r + k;
    const v8bf xhi = __builtin_bit_cast(v8bf, xh[u * (PC / 8) + g]);
    const v8bf xlo = __builtin_bit_cast(v8bf, xl[u * (PC / 8) + g]);
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
      acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xhi, W[ot][k], acc[ot], 0, 0, 0);
      acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xlo, W[ot][k], acc[ot], 0, 0, 0);
    }
  }
}

// max-pool of the lane's 4 positions, bias, ReLU (relu(max + b) equals the
// maximum of relu(. + b)); channel 16 ot + r of LDS row `row` as hi and lo
// halves; zeros instead where keep is false
__device__ __forceinline__ void pool4_store(const v4fp (&acc)[2], const float (&bo)[2], int r, int row, uint4* yh,
                                            uint4* yl, bool keep = true) {
#pragma unroll
  for (int ot = 0; ot < 2; ++ot) {
    const float m = fmaxf(fmaxf(acc[ot][0], acc[ot][1]), fmaxf(acc[ot][2], acc[ot][3]));
    const float y = keep ? fmaxf(m + bo[ot], 0.0f) : 0.0f;
    const unsigned short h = f_to_bf16(y);
    reinterpret_cast<unsigned short*>(yh)[row * PC + 16 * ot + r] = h;
    reinterpret_cast<unsigned short*>(yl)[row * PC + 16 * ot + r] = f_to_bf16(y - bf16_to_f(h));
  }
}

__device__ __forceinline__ void load_bias(const unsigned short* __restrict__ bias, int r, float (&bo)[2]) {
  bo[0] = bf16_to_f(bias[r]);
  bo[1] = bf16_to_f(bias[16 + r]);
}

constexpr int T1 = 128;          // layer-0 pooled outputs (layer-1 inputs) per tile
constexpr int NW = 8;            // waves per inference workgroup, one 16-position tile each in layer 1
constexpr int FB = PBLK + 40;    // the block's features with 20 zeros on either side
static_assert(T1 == 16 * NW, "one layer-1 tile per wave");

// SPEC false: features from feats, float[nb][4096]; SPEC true: computed here
// from bins 4096 b + t of the spectrum (n bins), as k_ps_features computes them.
// At most 128 VGPRs: two 8-wave workgroups per CU.
template <bool SPEC>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_ps_infer(
    const float* __restrict__ feats, const float2* __restrict__ spec, int64_t n, const unsigned short* __restrict__ w0,
    const unsigned short* __restrict__ b0, const uint4* __restrict__ pack, const unsigned short* __restrict__ b1,
    const unsigned short* __restrict__ b2, const unsigned short* __restrict__ b3, const unsigned short* __restrict__ wf,
    const unsigned short* __restrict__ bf, float* __restrict__ logits) {
  __shared__ unsigned short fh[FB], fl[FB];                         // features, hi and lo
  __shared__ uint4 xh[(T1 + 8) * PC / 8], xl[(T1 + 8) * PC / 8];  // layer-1 input tile, later a3
  __shared__ uint4 ah[(256 + 8) * PC / 8], al[(256 + 8) * PC / 8];  // a2, rows 4 .. 259
  __shared__ float hmax[4][PC];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g = lane >> 4, r = lane & 15;
  const float* f = SPEC ? nullptr : feats + (size_t)b * PBLK;
  const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
  if (tid < 32) {  // zero rows 0..3 and 260..263 of a2
    const int row = tid < 16 ? tid / 4 : 260 + (tid - 16) / 4;
    ah[row * 4 + (tid & 3)] = zero4;
    al[row * 4 + (tid & 3)] = zero4;
  }
  // layer 0: K = 32 holds the 9 taps twice (k and 16 + k), against the hi and
  // the lo half of the features, so one product gives 16 positions x 16
  // channels at FP32-level accuracy.  Lane (r, g) of the weight operand:
  // W_0[16 ot + r][8 (g % 2) + e], zero past tap 8.
  v8bf W0[2];
#pragma unroll
  for (int ot = 0; ot < 2; ++ot) {
    unsigned short a8[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = 8 * (g & 1) + e;
      a8[e] = k < PK ? w0[(16 * ot + r) * PK + k] : (unsigned short)0;
    }
    W0[ot] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(a8));
  }
  float bo0[2];
  load_bias(b0, r, bo0);
  v8bf W[2][PK];
  float bo[2];
  load_w(pack, 1, lane, W);
  load_bias(b1, r, bo);
  // the whole block's features: word e holds feature e - 20 (zero outside
  // the block and past the spectrum), every load issued before the first store
  const int64_t bin0 = (int64_t)b * PBLK;
  auto feature = [&](int t) {
    if (t < 0 || t >= PBLK) return 0.0f;
    if (!SPEC) return f[t];
    if (bin0 + t >= n) return 0.0f;
    const float2 c = spec[bin0 + t];
    return log1pf(c.x * c.x + c.y * c.y);
  };
  {
    constexpr int PER = (FB + 64 * NW - 1) / (64 * NW);
    float fv[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) fv[i] = feature(tid + 64 * NW * i - 20);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + 64 * NW * i;
      if (e < FB) {
        const unsigned short h = f_to_bf16(fv[i]);
        fh[e] = h;
        fl[e] = f_to_bf16(fv[i] - bf16_to_f(h));
      }
    }
  }
  for (int j = 0; j < 1024 / T1; ++j) {
    __syncthreads();  // the features are in; the previous tile is no longer read
    // tile row u is layer-1 input position T1 j - 4 + u; it pools layer-0
    // outputs 4 (T1 j - 4 + u) + q, q < 4, whose taps reach 4 before and 4 after
    // layer 0: (T1 + 8) / 4 tiles of 16 outputs; tile tt, row r is layer-0
    // position 4 T1 j - 16 + 16 tt + r, whose tap k reads feature word
    // 4 T1 j + 16 tt + r + k
    for (int tt = wv; tt < (T1 + 8) / 4; tt += NW) {
      const int base = 4 * T1 * j + 16 * tt + r;
      const unsigned short* src = g < 2 ? fh : fl;
      unsigned short b8[8];
      if ((g & 1) == 0) {
#pragma unroll
        for (int e = 0; e < 8; ++e) b8[e] = src[base + e];
      } else {
        b8[0] = src[base + 8];
#pragma unroll
        for (int e = 1; e < 8; ++e) b8[e] = 0;
      }
      const v8bf X = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(b8));
      v4fp acc[2];
#pragma unroll
      for (int ot = 0; ot < 2; ++ot)
        acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X, W0[ot], v4fp{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
      const int u = 4 * tt + g;  // pooled row, layer-1 input position T1 j - 4 + u
      const int pos = T1 * j - 4 + u;
      pool4_store(acc, bo0, r, u, xh, xl, pos >= 0 && pos < 1024);
    }
    __syncthreads();
    // layer 1: wave wv, positions T1 j + 16 wv + 4 g + v, pooled into a2 row T1 j / 4 + 4 wv + g + 4
    v4fp acc[2];
    mfma_tile(xh, xl, 16 * wv, W, r, g, acc);
    pool4_store(acc, bo, r, T1 * j / 4 + 4 * wv + g + 4, ah, al);
  }
  __syncthreads();
  if (tid < 32) {  // a3 in the tile buffer: zero rows 0..3 and 68..71
    const int row = tid < 16 ? tid / 4 : 68 + (tid - 16) / 4;
    xh[row * 4 + (tid & 3)] = zero4;
    xl[row * 4 + (tid & 3)] = zero4;
  }
  // layer 2: 16 tiles of 16 positions, pooled into a3 row 4 tt + g + 4
  load_w(pack, 2, lane, W);
  load_bias(b2, r, bo);
  for (int tt = wv; tt < 16; tt += NW) {
    v4fp acc[2];
    mfma_tile(ah, al, 16 * tt, W, r, g, acc);
    pool4_store(acc, bo, r, 4 * tt + g + 4, xh, xl);
  }
  __syncthreads();
  // layer 3 (waves 0..3): positions 16 wv + 4 g + v; the maximum over
  // positions, bias, ReLU
  if (wv < 4) {
    load_w(pack, 3, lane, W);
    load_bias(b3, r, bo);
    v4fp acc[2];
    mfma_tile(xh, xl, 16 * wv, W, r, g, acc);
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
      float m = fmaxf(fmaxf(acc[ot][0], acc[ot][1]), fmaxf(acc[ot][2], acc[ot][3]));
      m = fmaxf(m, __shfl_xor(m, 16));
      m = fmaxf(m, __shfl_xor(m, 32));
      if (g == 0) hmax[wv][16 * ot + r] = fmaxf(m + bo[ot], 0.0f);
    }
  }
  __syncthreads();
  if (tid == 0) {
    float lg = bf16_to_f(bf[0]);
    for (int c = 0; c < PC; ++c) {
      const float h = fmaxf(fmaxf(hmax[0][c], hmax[1][c]), fmaxf(hmax[2][c], hmax[3][c]));
      lg = fmaf(bf16_to_f(wf[c]), h, lg);
    }
    logits[b] = lg;
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
// Workgroup = (tile of PT positions, group of wgrad_group samples); each thread sums
// its (o, i) pairs (or, for one input channel, its pair over one of several
// position segments) in registers, then one atomic per weight.
// Samples per group: every workgroup adds its partial sums to the same
// weights, and float atomics on one address serialise in L2, so the
// one-channel layer (288 weights) takes larger groups.
template <int CIN>
constexpr int wgrad_group() {
  return CIN == 1 ? 16 : 4;
}
constexpr int XR = PT + 9;  // x row stride: odd, so the 32 input channels of a wave fall in distinct banks
template <int CIN>
__global__ __launch_bounds__(256) void k_ps_wgrad(const float* __restrict__ dz, const float* __restrict__ x, int L,
                                                  int nb, float* __restrict__ gw, float* __restrict__ gb) {
  constexpr int SG = wgrad_group<CIN>();
  __shared__ float xs[CIN][XR];
  __shared__ float ds[PC][PT];
  const int t0 = blockIdx.x * PT;
  const int b0 = blockIdx.y * SG;
  const int tid = threadIdx.x;
  const int T = min(PT, L - t0);  // a multiple of 8: L is 64, 256, 1024 or 4096
  constexpr int PAIRS = PC * CIN;
  constexpr int PPT = (PAIRS + 255) / 256;
  // fewer pairs than threads (CIN = 1): the threads of a pair split the positions
  constexpr int NSEG = PAIRS >= 256 ? 1 : 256 / PAIRS;
  static_assert(NSEG == 1 || PPT == 1, "either several pairs or several segments per thread");
  const int seg = NSEG == 1 ? 0 : tid / PAIRS;
  const int TS = NSEG == 1 ? T : ((T + NSEG - 1) / NSEG + 7) / 8 * 8;  // segment length, a multiple of 8
  const int tb0 = seg * TS, tb1 = min(T, tb0 + TS);
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
      const int pr = NSEG == 1 ? tid + 256 * u : tid % PAIRS;
      if (pr < PAIRS) {
        const int o = pr / CIN, i = pr % CIN;
        // 8 positions at a time from a 16-value window in registers (the sum
        // over t of each tap still runs in t order)
        for (int tb = tb0; tb < tb1; tb += 8) {
          float dv[8], xw[16];
#pragma unroll
          for (int q = 0; q < 8; ++q) dv[q] = ds[o][tb + q];
#pragma unroll
          for (int e = 0; e < 16; ++e) xw[e] = xs[i][tb + e];
#pragma unroll
          for (int q = 0; q < 8; ++q)
#pragma unroll
            for (int k = 0; k < PK; ++k) acc[u][k] = fmaf(dv[q], xw[q + k], acc[u][k]);
        }
      }
    }
    if (tid < PC)
      for (int t = 0; t < T; ++t) accb += ds[tid][t];
  }
  if (NSEG > 1) {
    // the segments' partial sums of each weight meet in LDS: one atomic per weight
    __shared__ float red[NSEG > 1 ? NSEG * PAIRS * PK : 1];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < PK; ++k) red[(seg * PAIRS + tid % PAIRS) * PK + k] = acc[0][k];
    __syncthreads();
    for (int w = tid; w < PAIRS * PK; w += 256) {
      float v = 0.0f;
      for (int q = 0; q < NSEG; ++q) v += red[q * PAIRS * PK + w];
      atomicAdd(&gw[w], v);  // w = (o * CIN + i) * PK + k with CIN = 1
    }
  } else {
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int pr = tid + 256 * u;
      if (pr < PAIRS) {
        const int o = pr / CIN, i = pr % CIN;
#pragma unroll
        for (int k = 0; k < PK; ++k) atomicAdd(&gw[((size_t)o * CIN + i) * PK + k], acc[u][k]);
      }
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
// closure of the flagged blocks as its list.  A NaN threshold or a logit that
// is not finite selects every block (the plain search).
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
  __shared__ int s_all;
  const int t = threadIdx.x;
  // Fallback to the plain search: a NaN threshold or any logit that is not
  // finite (a diverged or broken model) searches every block.
  if (t == 0) s_all = thr != thr ? 1 : 0;
  __syncthreads();
  for (int b = t; b < nblk; b += kSelThreads) {
    s_search[b] = 0;
    s_src[b] = 0;
    if (!(fabsf(logits[b]) <= 3.402823466e38f)) s_all = 1;  // NaN or +-inf
  }
  __syncthreads();
  for (int f = t; f < nblk; f += kSelThreads) {
    if (s_all) {
      s_search[f] = 1;
      continue;
    }
    if (!(logits[f] > thr)) continue;
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
  if (!train) {
    // inference: the whole network per sample in one kernel, logits only
    hipLaunchKernelGGL(k_ps_infer<false>, dim3(nb), dim3(64 * NW), 0, s, feats, nullptr, (int64_t)0, w + ps_off_w(0),
                       w + ps_off_b(0),
                       reinterpret_cast<const uint4*>(pb.wpack), w + ps_off_b(1), w + ps_off_b(2), w + ps_off_b(3),
                       w + ps_off_fc(), w + ps_off_fc() + PC, logits);
    return hipGetLastError();
  }
  // training forward on the vector units, recording the activations and the
  // max-pool positions for the backward pass
  hipLaunchKernelGGL((k_ps_conv<1, 0>), dim3(PBLK / PT, nb), blk, 0, s, feats, PBLK, w + ps_off_w(0),
                     w + ps_off_b(0), 4, pb.a1, pb.arg1, nullptr, nullptr);
  hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1024 / PT, nb), blk, 0, s, pb.a1, 1024, w + ps_off_w(1),
                     w + ps_off_b(1), 4, pb.a2, pb.arg2, nullptr, nullptr);
  hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1, nb), blk, 0, s, pb.a2, 256, w + ps_off_w(2), w + ps_off_b(2), 4,
                     pb.a3, pb.arg3, nullptr, nullptr);
  hipLaunchKernelGGL((k_ps_conv<PC, 0>), dim3(1, nb), blk, 0, s, pb.a3, 64, w + ps_off_w(3), w + ps_off_b(3), 1,
                     pb.r4, nullptr, nullptr, nullptr);
  hipLaunchKernelGGL(k_ps_head, dim3(nb), dim3(64), 0, s, pb.r4, w + ps_off_fc(), w + ps_off_fc() + PC, labels,
                     pos_weight, nb, logits, loss, pb.dz4, pb.grad + ps_off_fc());
  // backward: weight gradients of layer 4, then the data gradient into dz3, ...
  const unsigned g1 = (unsigned)((nb + wgrad_group<1>() - 1) / wgrad_group<1>());
  const unsigned g32 = (unsigned)((nb + wgrad_group<PC>() - 1) / wgrad_group<PC>());
  hipLaunchKernelGGL(k_ps_wgrad<PC>, dim3(1, g32), blk, 0, s, pb.dz4, pb.a3, 64, nb, pb.grad + ps_off_w(3),
                     pb.grad + ps_off_b(3));
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
      hipLaunchKernelGGL(k_ps_wgrad<1>, dim3(4 * L / PT, g1), blk, 0, s, dz_below[0], xin[0], 4 * L, nb,
                         pb.grad + ps_off_w(0), pb.grad + ps_off_b(0));
    else
      hipLaunchKernelGGL(k_ps_wgrad<PC>, dim3(4 * L / PT, g32), blk, 0, s, dz_below[l - 1], xin[l - 1], 4 * L, nb,
                         pb.grad + ps_off_w(l - 1), pb.grad + ps_off_b(l - 1));
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

hipError_t ps_infer_spectrum(const PsBuffers& pb, const float2* x, int64_t n, int nb, float* logits, hipStream_t s) {
  const unsigned short* w = pb.wbf;
  hipLaunchKernelGGL(k_ps_infer<true>, dim3(nb), dim3(64 * NW), 0, s, nullptr, x, n, w + ps_off_w(0), w + ps_off_b(0),
                     reinterpret_cast<const uint4*>(pb.wpack), w + ps_off_b(1), w + ps_off_b(2), w + ps_off_b(3),
                     w + ps_off_fc(), w + ps_off_fc() + PC, logits);
  return hipGetLastError();
}

// the inference kernel's A operands follow every change of the BF16 weights
static hipError_t ps_pack(const PsBuffers& pb, hipStream_t s) {
  const unsigned short* w = pb.wbf;
  hipLaunchKernelGGL(k_ps_pack, dim3((kPackWords + 255) / 256), dim3(256), 0, s, w + ps_off_w(1), w + ps_off_w(2),
                     w + ps_off_w(3), reinterpret_cast<uint4*>(pb.wpack));
  return hipGetLastError();
}

hipError_t ps_adam(const PsBuffers& pb, float lr, float b1, float b2, float c1, float c2, float eps, hipStream_t s) {
  const int np = ps_param_count();
  hipLaunchKernelGGL(k_ps_adam, dim3((np + 255) / 256), dim3(256), 0, s, pb.theta, pb.grad, pb.m, pb.v, pb.wbf, np, lr,
                     b1, b2, c1, c2, eps);
  return ps_pack(pb, s);
}

hipError_t ps_round(const PsBuffers& pb, hipStream_t s) {
  const int np = ps_param_count();
  hipLaunchKernelGGL(k_ps_round, dim3((np + 255) / 256), dim3(256), 0, s, pb.theta, pb.wbf, np);
  return ps_pack(pb, s);
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
