// Harmonic summing with threshold detection and candidate compaction
// (Section 2.2, Algorithm 1), all harmonic planes at once without storing
// them (the MultipleHP organisation of Section 2.2).
//
//   HP_1(i, j) = FOP(i, j)
//   HP_k(i, j) = HP_{k-1}(i, j) + FOP(trunc(i/k), floor(j/k)),  k = 2..NH
//   a cell with HP_k(i, j) > TA(k, i) is appended to list k.
//
// Sums are FP32 in k order (no reassociation, no contraction: there are only
// additions), so every kernel here is bit-identical to a sequential FP32 sum.
// In the stretch-map kernels each thread owns 4 adjacent columns j0..j0+3;
// for k >= 2 those columns read at most two adjacent source columns
// (floor(j/k) spans <= 2 values).  The kernels of the other index maps
// interleave a thread's columns across the wave instead (see there).

#include "fdas_internal.h"

namespace fdas {
namespace {

constexpr int HS_THREADS = 256;

// Appends one record to list k.  A plan keeps (2 z_max + 1) n_max below 2^31,
// so a count cannot wrap; the unsigned compare still keeps any slot that is
// not in [0, cap) from being written.
__device__ __forceinline__ void emit(int k, int i, int j, float p, fdas_cand* __restrict__ cands, int cap,
                                     int32_t* __restrict__ counts) {
  const int slot = atomicAdd(&counts[k - 1], 1);
  if ((unsigned)slot < (unsigned)cap) {
    int4 rec = make_int4(k, i, j, __float_as_int(p));
    *reinterpret_cast<int4*>(cands + (size_t)(k - 1) * cap + slot) = rec;
  }
}

// ---------------------------------------------------------------------------
// Generic path (any row count): runtime row loop; a source value of harmonic k
// is fetched once per change of trunc(i/k) and kept across the k rows sharing it.
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

// ---------------------------------------------------------------------------
// Alternative index maps (plan option hsum_index), any row count.  A pulsar
// whose fundamental sits at (z, r) has its m-th harmonic at (m z, m r).
//
// Both kernels take a column tile of XT = 4 * HS_THREADS columns per
// workgroup (tile from tile_of_block when given, else blockIdx.x) and give
// thread t the columns tile * XT + t + HS_THREADS * a, a = 0..3, so that a
// wave's load of one source row covers 64 consecutive output columns: 64
// consecutive source columns for the fundamental, 64 at stride m for FOP(k i,
// k j), 64 nearly consecutive ones (stretch factor <= 1) for rho(m j, k).
// Candidates are appended with one atomic per wave and plane (hits are rare;
// a dense plane still costs one reservation per wave).

constexpr int XT = 4 * HS_THREADS;

// Lane offsets inside the wave from ballots of each lane's 3-bit hit count;
// the lowest active lane reserves the wave's slots in list m.  Every lane of
// the wave calls this with the same m (the caller is wave-uniform).
__device__ __forceinline__ void wave_append(int m, int i, const int (&col)[4], const float (&v)[4], unsigned bits,
                                            fdas_cand* __restrict__ cands, int cap, int32_t* __restrict__ counts) {
  const int c = __popc(bits);
  const unsigned long long b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4);
  const int total = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
  if (total == 0) return;  // uniform
  auto below = [](unsigned long long b) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
  };
  const int mine = below(b0) + 2 * below(b1) + 4 * below(b2);
  const unsigned long long act = __ballot(1);
  const int lead = (int)__builtin_ctzll(act);
  int base = 0;
  if ((int)(threadIdx.x & 63) == lead) base = atomicAdd(&counts[m - 1], total);
  int slot = __shfl(base, lead) + mine;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    if ((bits >> a) & 1u) {
      if ((unsigned)slot < (unsigned)cap)
        *reinterpret_cast<int4*>(cands + (size_t)(m - 1) * cap + slot) = make_int4(m, i, col[a], __float_as_int(v[a]));
      ++slot;
    }
  }
}

// Tile of this workgroup (-1: none) and the thread's four columns.
__device__ __forceinline__ int xt_tile(const int* __restrict__ tile_of_block, int n) {
  const int tile = tile_of_block ? tile_of_block[blockIdx.x] : (int)blockIdx.x;
  return (tile >= 0 && (int64_t)tile * XT < n) ? tile : -1;
}

// Raw buffer resource over part of one FOP row: loads at byte offsets >=
// bytes read 0 (the hardware range check), so columns past n - 1 need no
// compare.  The resource starts at the first column a workgroup reads, so
// offsets stay below 32 KB whatever n is.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const float* base, int64_t cols_left) {
  const uint32_t bytes = cols_left <= 0 ? 0u : (cols_left >= 16384 ? 65536u : (uint32_t)cols_left * 4u);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float row_load(__amdgpu_buffer_rsrc_t rs, int byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, byte_off, 0, 0));
}

// Fundamental-anchored: HP_k(i, j) = HP_{k-1}(i, j) + FOP(k i, k j), a term
// being 0 where (k i, k j) is outside the plane.  Cumulative in k.  A row's
// loads (the fundamental and every harmonic's source row k i inside the
// plane) are issued together before its sums, as buffer loads whose range
// check supplies the zeros of columns k j >= n.  Harmonic m of the tile
// starting at column t0 reads columns m t0 + m (t + 256 a).  Six waves per
// SIMD (80 VGPRs) hide the load latency best: 0.94 ms on a 2^22 plane against
// 0.98 ms at five and 1.00 ms at eight (with spills); loading row r + 1
// before the sums of row r (three waves) took 1.06 ms.
template <int NH>
__global__ __launch_bounds__(HS_THREADS, 6) void k_harmsum_fund(const float* __restrict__ fop, int64_t ld, int n,
                                                             int z_max, const int* __restrict__ tile_of_block,
                                                             const float* __restrict__ ta,
                                                             fdas_cand* __restrict__ cands, int cap,
                                                             int32_t* __restrict__ counts) {
  const int tile = xt_tile(tile_of_block, n);
  if (tile < 0) return;  // uniform
  const int rows = 2 * z_max + 1;
  const int64_t t0 = (int64_t)tile * XT;
  const int t = (int)threadIdx.x;
  int col[4];
  bool in[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    col[a] = (int)t0 + t + HS_THREADS * a;  // n <= 2^30, so no wrap
    in[a] = col[a] < n;
  }
  for (int r = 0; r < rows; ++r) {
    const int i = r - z_max;
    float v[NH + 1][4];
    {
      const __amdgpu_buffer_rsrc_t rs = row_rsrc(fop + (size_t)r * ld + t0, (int64_t)n - t0);
#pragma unroll
      for (int a = 0; a < 4; ++a) v[1][a] = row_load(rs, 4 * (t + HS_THREADS * a));
    }
#pragma unroll
    for (int m = 2; m <= NH; ++m) {
      const int si = m * i;
      if (si >= -z_max && si <= z_max) {  // uniform
        const __amdgpu_buffer_rsrc_t rs =
            row_rsrc(fop + (size_t)(si + z_max) * ld + m * t0, (int64_t)n - m * t0);
#pragma unroll
        for (int a = 0; a < 4; ++a) v[m][a] = row_load(rs, 4 * m * (t + HS_THREADS * a));
      } else {
#pragma unroll
        for (int a = 0; a < 4; ++a) v[m][a] = 0.0f;
      }
    }
    float hp[4];
#pragma unroll
    for (int m = 1; m <= NH; ++m) {
      const float th = ta[(m - 1) * rows + r];
      unsigned bits = 0u;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        hp[a] = m == 1 ? v[1][a] : hp[a] + v[m][a];
        bits |= (in[a] && hp[a] > th) ? 1u << a : 0u;
      }
      wave_append(m, i, col, hp, bits, cands, cap, counts);
    }
  }
}

// Highest-harmonic-anchored: HP_k(i, j) = sum_{m=1..k} FOP(rho(m i, k), rho(m j, k)),
// summed in m order, rho = rounding to the nearest integer with halves away
// from zero.  Every index is inside the plane; the planes are not cumulative.
//
// rho(m x, k) depends on m/k only, so the terms of all k <= NH read one value
// per reduced fraction p/q (q <= NH): 22 fractions for NH = 8.  Each
// fraction's four values stay in registers while its source row rho(p i, q)
// is unchanged (it changes on about p/q of the rows).

__host__ __device__ constexpr int gcd_c(int a, int b) { return b == 0 ? a : gcd_c(b, a % b); }

// reduced fractions p/q, 1 <= p <= q <= nh, ordered by q, then p
__host__ __device__ constexpr int frac_count(int nh) {
  int c = 0;
  for (int q = 1; q <= nh; ++q)
    for (int p = 1; p <= q; ++p) c += gcd_c(p, q) == 1 ? 1 : 0;
  return c;
}
__host__ __device__ constexpr int frac_index(int m, int k) {
  const int g = gcd_c(m, k), p = m / g, q = k / g;
  int idx = frac_count(q - 1);
  for (int pp = 1; pp < p; ++pp) idx += gcd_c(pp, q) == 1 ? 1 : 0;
  return idx;
}
__host__ __device__ constexpr int frac_num(int idx) {
  for (int q = 1;; ++q)
    for (int p = 1; p <= q; ++p)
      if (gcd_c(p, q) == 1 && idx-- == 0) return p;
}
__host__ __device__ constexpr int frac_den(int idx) {
  for (int q = 1;; ++q)
    for (int p = 1; p <= q; ++p)
      if (gcd_c(p, q) == 1 && idx-- == 0) return q;
}
static_assert(frac_count(8) == 22 && frac_index(4, 8) == 1 && frac_num(5) == 3 && frac_den(5) == 4, "fractions");

template <int NH>
struct HighState {
  float val[frac_count(NH)][4];
  int row[frac_count(NH)];  // source row the values belong to (uniform)
};

// rho(P x, Q) for x >= 0.  Narrow: 2 P x + Q < 2^32 (n * 2 NH < 2^32).  Wide,
// any x < 2^31: with x = Q u + w (w < Q), P x / Q = P u + P w / Q, so the
// rounding only involves P w < P Q.
template <int P, int Q, bool WIDE>
__device__ __forceinline__ int rho_pos(int x) {
  if constexpr (WIDE) {
    const unsigned u = (unsigned)x / Q, w = (unsigned)x - u * Q;
    return (int)(P * u + (2u * P * w + Q) / (2u * Q));
  } else {
    return (int)((2u * P * (unsigned)x + Q) / (2u * Q));
  }
}

// refresh fraction F and the ones after it for output row i
template <int NH, bool WIDE, int F>
__device__ __forceinline__ void hi_refresh(HighState<NH>& st, const float* __restrict__ fop, int64_t ld, int z_max,
                                           int i, const int (&colc)[4]) {
  if constexpr (F < frac_count(NH)) {
    constexpr int P = frac_num(F), Q = frac_den(F);
    const int s = rho_pos<P, Q, false>(i < 0 ? -i : i);
    const int srow = (i < 0 ? -s : s) + z_max;
    if (srow != st.row[F]) {  // uniform
      st.row[F] = srow;
      const float* src = fop + (size_t)srow * ld;
#pragma unroll
      for (int a = 0; a < 4; ++a) st.val[F][a] = src[rho_pos<P, Q, WIDE>(colc[a])];
    }
    hi_refresh<NH, WIDE, F + 1>(st, fop, ld, z_max, i, colc);
  }
}

// HP_K = terms m = 1..K in m order
template <int NH, int K, int M>
__device__ __forceinline__ void hi_sum(const HighState<NH>& st, float (&hp)[4]) {
  if constexpr (M <= K) {
    constexpr int FI = frac_index(M, K);
#pragma unroll
    for (int a = 0; a < 4; ++a) hp[a] = M == 1 ? st.val[FI][a] : hp[a] + st.val[FI][a];
    hi_sum<NH, K, M + 1>(st, hp);
  }
}

template <int NH, int K>
__device__ __forceinline__ void hi_planes(const HighState<NH>& st, int r, int i, int rows, const int (&col)[4],
                                          const bool (&in)[4], const float* __restrict__ ta,
                                          fdas_cand* __restrict__ cands, int cap, int32_t* __restrict__ counts) {
  if constexpr (K <= NH) {
    float hp[4];
    hi_sum<NH, K, 1>(st, hp);
    const float t = ta[(K - 1) * rows + r];
    unsigned bits = 0u;
#pragma unroll
    for (int a = 0; a < 4; ++a) bits |= (in[a] && hp[a] > t) ? 1u << a : 0u;
    wave_append(K, i, col, hp, bits, cands, cap, counts);
    hi_planes<NH, K + 1>(st, r, i, rows, col, in, ta, cands, cap, counts);
  }
}

template <int NH, bool WIDE>
__global__ __launch_bounds__(HS_THREADS) void k_harmsum_high(const float* __restrict__ fop, int64_t ld, int n,
                                                             int z_max, const int* __restrict__ tile_of_block,
                                                             const float* __restrict__ ta,
                                                             fdas_cand* __restrict__ cands, int cap,
                                                             int32_t* __restrict__ counts) {
  const int tile = xt_tile(tile_of_block, n);
  if (tile < 0) return;  // uniform
  const int rows = 2 * z_max + 1;
  int col[4], colc[4];
  bool in[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    col[a] = tile * XT + (int)threadIdx.x + HS_THREADS * a;
    in[a] = col[a] < n;
    colc[a] = in[a] ? col[a] : n - 1;  // columns past n - 1 read column n - 1 and are never emitted
  }
  constexpr int NF = frac_count(NH);
  HighState<NH> st;
#pragma unroll
  for (int f = 0; f < NF; ++f) st.row[f] = -1;
  for (int r = 0; r < rows; ++r) {
    const int i = r - z_max;
    hi_refresh<NH, WIDE, 0>(st, fop, ld, z_max, i, colc);
    hi_planes<NH, 1>(st, r, i, rows, col, in, ta, cands, cap, counts);
  }
}

// ---------------------------------------------------------------------------
// Fast path for a compile-time row count (2*Z+1 rows), in two phases.
//
// Phase 1 (k_harmsum_z): each thread owns 4 adjacent columns and walks all
// rows.  Rows and harmonics are unrolled at compile time (template
// recursion), so every source row and register slot is a constant.  Loads are
// issued DEPTH rows ahead of their use: the unstretched row r+DEPTH, and for
// each k >= 2 the source row trunc((r+DEPTH-Z)/k) when it first appears.  A
// row costs 4*(NH-1) adds plus one max-reduction and compare per harmonic; the
// thread only records which of its rows hold a cell above threshold (a bit
// mask), and a block appends one entry {j0, mask} per thread with hits to a
// global list.
//
// Phase 2 (k_harmsum_emit): a grid-stride kernel gives every (entry, row) with
// its bit set to one thread, which re-forms that row's sums from memory in the
// same k order (bit-identical to phase 1) and appends the candidates.  Hits
// cluster around strong pulsars, so spreading them over the whole GPU keeps a
// few dense tiles from serialising the kernel.
//
// Source columns of the 4 columns j0..j0+3 (j0 = 4g) for harmonic k:
//   k = 2:        (j0/2, j0/2, j0/2+1, j0/2+1)        -- fixed pattern
//   k = 4, 8:     j0/k for all four (j0 mod k + 3 < k)
//   k = 3,5,6,7:  column a reads j0/k + 1 iff (j0 mod k) + a >= k

constexpr int DEPTH = 8;
constexpr int RING = DEPTH / 2 + 3;  // > source rows of one harmonic first used within DEPTH rows

__host__ __device__ constexpr int src_row(int r, int m, int Z) { return (r - Z) / m + Z; }  // C truncation
__host__ __device__ constexpr int slot_of(int r, int m, int Z) { return (src_row(r, m, Z) - src_row(0, m, Z)) % RING; }
__host__ __device__ constexpr bool starts(int r, int m, int Z) {
  return r == 0 || src_row(r, m, Z) != src_row(r - 1, m, Z);
}
__host__ __device__ constexpr bool needs_hi(int m) { return m != 4 && m != 8; }

template <int NH>
struct HsState {
  float4 ring1[DEPTH];
  float lo_ring[NH + 1][RING];
  float hi_ring[NH + 1][RING];
  float val[NH + 1][4];
  unsigned hitmask[3];
};

// loads of the stretched source rows first needed at row R
template <int Z, int NH, int R, int M>
__device__ __forceinline__ void hs_issue_m(HsState<NH>& st, const float* __restrict__ fop, int64_t ld,
                                           const int (&lo)[NH + 1]) {
  if constexpr (M <= NH) {
    if constexpr (starts(R, M, Z)) {
      constexpr int S = src_row(R, M, Z);
      constexpr int SL = slot_of(R, M, Z);
      const float* src = fop + (size_t)S * ld + lo[M];
      if constexpr (M == 2) {
        const float2 q = *reinterpret_cast<const float2*>(src);  // j0/2 is even
        st.lo_ring[M][SL] = q.x;
        st.hi_ring[M][SL] = q.y;
      } else {
        st.lo_ring[M][SL] = src[0];
        if constexpr (needs_hi(M)) st.hi_ring[M][SL] = src[1];
      }
    }
    hs_issue_m<Z, NH, R, M + 1>(st, fop, ld, lo);
  }
}

template <int Z, int NH, int R>
__device__ __forceinline__ void hs_issue(HsState<NH>& st, const float* __restrict__ fop, int64_t ld, int j0,
                                         const int (&lo)[NH + 1]) {
  if constexpr (R < 2 * Z + 1) {
    st.ring1[R % DEPTH] = *reinterpret_cast<const float4*>(fop + (size_t)R * ld + j0);
    hs_issue_m<Z, NH, R, 2>(st, fop, ld, lo);
  }
}

template <int Z, int NH, int R, int M>
__device__ __forceinline__ void hs_harm(HsState<NH>& st, float (&hp)[4], bool& hit, const int (&rmod)[NH + 1],
                                        const float* __restrict__ s_ta) {
  if constexpr (M <= NH) {
    if constexpr (starts(R, M, Z)) {
      constexpr int SL = slot_of(R, M, Z);
      const float vl = st.lo_ring[M][SL];
      if constexpr (M == 2) {
        const float vh = st.hi_ring[M][SL];
        st.val[M][0] = vl;
        st.val[M][1] = vl;
        st.val[M][2] = vh;
        st.val[M][3] = vh;
      } else if constexpr (!needs_hi(M)) {
#pragma unroll
        for (int a = 0; a < 4; ++a) st.val[M][a] = vl;
      } else {
        const float vh = st.hi_ring[M][SL];
        st.val[M][0] = vl;
#pragma unroll
        for (int a = 1; a < 4; ++a) st.val[M][a] = (rmod[M] + a >= M) ? vh : vl;
      }
    }
    const float t = s_ta[R * 8 + (M - 1)];
#pragma unroll
    for (int a = 0; a < 4; ++a) hp[a] = hp[a] + st.val[M][a];
    // one compare per harmonic: any of the 4 columns above threshold (NaN never is)
    hit = hit || fmaxf(fmaxf(hp[0], hp[1]), fmaxf(hp[2], hp[3])) > t;
    hs_harm<Z, NH, R, M + 1>(st, hp, hit, rmod, s_ta);
  }
}

template <int Z, int NH, int R>
__device__ __forceinline__ void hs_rows(HsState<NH>& st, const float* __restrict__ fop, int64_t ld, int j0,
                                        const int (&lo)[NH + 1], const int (&rmod)[NH + 1],
                                        const float* __restrict__ s_ta) {
  // take row R out of its ring slot before the slot is refilled with row R + DEPTH
  const float4 v = st.ring1[R % DEPTH];
  hs_issue<Z, NH, R + DEPTH>(st, fop, ld, j0, lo);
  float hp[4] = {v.x, v.y, v.z, v.w};
  bool hit = fmaxf(fmaxf(hp[0], hp[1]), fmaxf(hp[2], hp[3])) > s_ta[R * 8];
  hs_harm<Z, NH, R, 2>(st, hp, hit, rmod, s_ta);
  st.hitmask[R / 32] |= hit ? (1u << (R % 32)) : 0u;
  // Keep the software pipeline as written: the row's sums are consumed here
  // (an empty asm that reads and rewrites the hit word), and no instruction
  // crosses the row boundary.
  __asm__ volatile("" : "+v"(st.hitmask[R / 32]));
  __builtin_amdgcn_sched_barrier(0);
  if constexpr (R + 1 < 2 * Z + 1) hs_rows<Z, NH, R + 1>(st, fop, ld, j0, lo, rmod, s_ta);
}

template <int Z, int NH, int R>
__device__ __forceinline__ void hs_prologue(HsState<NH>& st, const float* __restrict__ fop, int64_t ld, int j0,
                                            const int (&lo)[NH + 1]) {
  hs_issue<Z, NH, R>(st, fop, ld, j0, lo);
  if constexpr (R + 1 < DEPTH) hs_prologue<Z, NH, R + 1>(st, fop, ld, j0, lo);
}

// Phase 1 over all columns [0, n) in groups of 4 (the last group may be
// partial).  The 16-byte read of the last group stays inside the row because
// ld >= n and ld % 4 == 0; a source column j/k + 1 read for k >= 2 is at most
// (n-1)/2 + 1 <= ld - 1.  Values read beyond column n - 1 only reach columns
// >= n, which phase 2 never emits.
// Phase 1 for one thread: columns j0..j0+3 of a plane with n columns.
// Returns the bit mask of rows holding a cell above threshold (3 words).
template <int Z, int NH>
__device__ __forceinline__ void hs_phase1_thread(const float* __restrict__ fop, int64_t ld, int j0,
                                                 const float* __restrict__ s_ta, unsigned (&mask)[3]) {
  int lo[NH + 1], rmod[NH + 1];
#pragma unroll
  for (int m = 0; m <= NH; ++m) {
    lo[m] = m >= 2 ? j0 / m : 0;
    rmod[m] = m >= 2 ? j0 - lo[m] * m : 0;
  }
  HsState<NH> st;
  st.hitmask[0] = st.hitmask[1] = st.hitmask[2] = 0u;
  hs_prologue<Z, NH, 0>(st, fop, ld, j0, lo);
  hs_rows<Z, NH, 0>(st, fop, ld, j0, lo, rmod, s_ta);
  mask[0] = st.hitmask[0];
  mask[1] = st.hitmask[1];
  mask[2] = st.hitmask[2];
}

template <int Z, int NH>
__device__ __forceinline__ void hs_load_ta(const float* __restrict__ ta, float* __restrict__ s_ta) {
  constexpr int ROWS = 2 * Z + 1;
  for (int e = threadIdx.x; e < ROWS * 8; e += blockDim.x) {
    const int r = e / 8, m = e % 8;
    s_ta[e] = m < NH ? ta[m * ROWS + r] : 0.0f;
  }
}

// Append this block's entries {j0, mask words} to the global hit-row list.
__device__ __forceinline__ void hs_flush_entries(const int4* __restrict__ s_ent, int cnt, int* s_base,
                                                 int4* __restrict__ hitrows, int32_t* __restrict__ hitrow_count) {
  if (cnt == 0) return;  // uniform
  if (threadIdx.x == 0) *s_base = atomicAdd(hitrow_count, cnt);
  __syncthreads();
  if (threadIdx.x < cnt) hitrows[*s_base + threadIdx.x] = s_ent[threadIdx.x];
}

// Phase 1 over all columns [0, n) in groups of 4 (the last group may be
// partial).  The 16-byte read of the last group stays inside the row because
// ld >= n and ld % 4 == 0; a source column j/k + 1 read for k >= 2 is at most
// (n-1)/2 + 1 <= ld - 1.  Values read beyond column n - 1 only reach columns
// >= n, which phase 2 never emits.
template <int Z, int NH, int TH = HS_THREADS>
__global__ __launch_bounds__(TH) void k_harmsum_z(const float* __restrict__ fop, int64_t ld, int n,
                                                          const int* __restrict__ tile_of_block,
                                                          const float* __restrict__ ta, int4* __restrict__ hitrows,
                                                          int32_t* __restrict__ hitrow_count) {
  constexpr int ROWS = 2 * Z + 1;
  static_assert(ROWS <= 96, "hit mask holds 96 rows");
  __shared__ float s_ta[ROWS * 8];  // [row][k-1]
  __shared__ int4 s_ent[TH];
  __shared__ int s_nent, s_base;
  hs_load_ta<Z, NH>(ta, s_ta);
  if (threadIdx.x == 0) s_nent = 0;
  __syncthreads();
  const int groups = (n + 3) / 4;
  const int tile = tile_of_block[blockIdx.x];  // -1: no tile for this block
  const int g = tile * TH + threadIdx.x;
  if (tile >= 0 && g < groups) {
    const int j0 = 4 * g;
    unsigned mask[3];
    hs_phase1_thread<Z, NH>(fop, ld, j0, s_ta, mask);
    if (mask[0] | mask[1] | mask[2]) {
      const int pos = atomicAdd(&s_nent, 1);
      s_ent[pos] = make_int4(j0, (int)mask[0], (int)mask[1], (int)mask[2]);
    }
  }
  __syncthreads();
  hs_flush_entries(s_ent, s_nent, &s_base, hitrows, hitrow_count);
}

// Batch form: workgroup blk_begin + blockIdx.x belongs to the last trial whose
// block0 is <= it; its tile comes from that trial's tile order.  Entries carry
// the trial in bits 21..31 of the third mask word (rows 64..84 use bits 0..20).
template <int Z, int NH, int TH>
__global__ __launch_bounds__(TH) void k_harmsum_z_batch(const HsTrial* __restrict__ trials, int ntrials,
                                                                int blk_begin, const float* __restrict__ ta,
                                                                int4* __restrict__ hitrows,
                                                                int32_t* __restrict__ hitrow_count) {
  constexpr int ROWS = 2 * Z + 1;
  static_assert(ROWS <= 85, "the trial tag uses bits 21..31 of the third mask word");
  __shared__ float s_ta[ROWS * 8];
  __shared__ int4 s_ent[TH];
  __shared__ int s_nent, s_base;
  hs_load_ta<Z, NH>(ta, s_ta);
  if (threadIdx.x == 0) s_nent = 0;
  __syncthreads();
  const int b = blk_begin + (int)blockIdx.x;
  int lo = 0, hi = ntrials - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (trials[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  const HsTrial tr = trials[lo];
  const int groups = (tr.n + 3) / 4;
  const int lb = b - tr.block0;
  const int tile = lb < tr.nblocks ? tr.tile_of_block[lb] : -1;
  const int g = tile * TH + threadIdx.x;
  if (tile >= 0 && g < groups) {
    const int j0 = 4 * g;
    unsigned mask[3];
    hs_phase1_thread<Z, NH>(tr.fop, tr.ld, j0, s_ta, mask);
    if (mask[0] | mask[1] | mask[2]) {
      const int pos = atomicAdd(&s_nent, 1);
      s_ent[pos] = make_int4(j0, (int)mask[0], (int)mask[1], (int)(mask[2] | ((unsigned)lo << 21)));
    }
  }
  __syncthreads();
  hs_flush_entries(s_ent, s_nent, &s_base, hitrows, hitrow_count);
}

// Phase 2 for one (entry, row): re-form the row's sums from memory in the
// same k order as phase 1 (bit-identical) and append its candidates.  Every
// column index read stays < ld (same bound as phase 1).
template <int Z, int NH>
__device__ __forceinline__ void hs_emit_row(const float* __restrict__ fop, int64_t ld, int n, int j0, int r,
                                            const float* __restrict__ ta, fdas_cand* __restrict__ cands, int cap,
                                            int32_t* __restrict__ counts) {
  constexpr int ROWS = 2 * Z + 1;
  const int i = r - Z;
  // all loads first (independent), then the sums in k order
  const float4 v = *reinterpret_cast<const float4*>(fop + (size_t)r * ld + j0);
  float src[NH + 1][4];
#pragma unroll
  for (int m = 2; m <= NH; ++m) {
    const float* rowp = fop + (size_t)(i / m + Z) * ld;
#pragma unroll
    for (int a = 0; a < 4; ++a) src[m][a] = rowp[(j0 + a) / m];
  }
  float hk[NH + 1][4];
  hk[1][0] = v.x;
  hk[1][1] = v.y;
  hk[1][2] = v.z;
  hk[1][3] = v.w;
#pragma unroll
  for (int m = 2; m <= NH; ++m)
#pragma unroll
    for (int a = 0; a < 4; ++a) hk[m][a] = hk[m - 1][a] + src[m][a];
  // reserve per plane, then write
#pragma unroll
  for (int m = 1; m <= NH; ++m) {
    const float t = ta[(m - 1) * ROWS + r];
    int c = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) c += (j0 + a < n && hk[m][a] > t) ? 1 : 0;
    if (c) {
      int slot = atomicAdd(&counts[m - 1], c);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        if (j0 + a < n && hk[m][a] > t) {
          if ((unsigned)slot < (unsigned)cap)
            *reinterpret_cast<int4*>(cands + (size_t)(m - 1) * cap + slot) =
                make_int4(m, i, j0 + a, __float_as_int(hk[m][a]));
          ++slot;
        }
      }
    }
  }
}

// Phase 2 for one wave: every active lane re-forms the sums of its row r of
// columns j0..j0+3 (same k order as phase 1, so bit-identical) and the wave
// appends the candidates of all lanes to one plane set (fop, cands, counts
// uniform across the wave).  Each plane's slots are reserved for the whole
// wave in one round of atomics: lane m - 1 reserves plane m, lane offsets come
// from ballots of the 3-bit per-lane counts.
template <int Z, int NH>
__device__ __forceinline__ void hs_emit_wave(const float* __restrict__ fop, int64_t ld, int n, int j0, int r,
                                             bool act, const float* __restrict__ ta,
                                             fdas_cand* __restrict__ cands, int cap,
                                             int32_t* __restrict__ counts, int lane) {
  constexpr int ROWS = 2 * Z + 1;
  const int i = r - Z;
  float hk[NH + 1][4];
  if (act) {
    const float4 v = *reinterpret_cast<const float4*>(fop + (size_t)r * ld + j0);
    float src[NH + 1][4];
#pragma unroll
    for (int m = 2; m <= NH; ++m) {
      const float* rowp = fop + (size_t)(i / m + Z) * ld;
#pragma unroll
      for (int a = 0; a < 4; ++a) src[m][a] = rowp[(j0 + a) / m];
    }
    hk[1][0] = v.x;
    hk[1][1] = v.y;
    hk[1][2] = v.z;
    hk[1][3] = v.w;
#pragma unroll
    for (int m = 2; m <= NH; ++m)
#pragma unroll
      for (int a = 0; a < 4; ++a) hk[m][a] = hk[m - 1][a] + src[m][a];
  }
  unsigned hits = 0u;  // bit 4 * (m - 1) + a: column j0 + a is a candidate of plane m
  int below_m[NH + 1], total[NH + 1];
  auto below = [&](unsigned long long b) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)b, 0u));
  };
  int mine = 0;
#pragma unroll
  for (int m = 1; m <= NH; ++m) {
    int c = 0;
    const float t = act ? ta[(m - 1) * ROWS + r] : 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const bool h = act && j0 + a < n && hk[m][a] > t;
      hits |= h ? 1u << (4 * (m - 1) + a) : 0u;
      c += h ? 1 : 0;
    }
    const unsigned long long b0 = __ballot(c & 1), b1 = __ballot(c & 2), b2 = __ballot(c & 4);
    total[m] = __popcll(b0) + 2 * __popcll(b1) + 4 * __popcll(b2);
    below_m[m] = below(b0) + 2 * below(b1) + 4 * below(b2);
    if (lane == m - 1) mine = total[m];
  }
  int base = 0;
  if (lane < NH && mine > 0) base = atomicAdd(&counts[lane], mine);
#pragma unroll
  for (int m = 1; m <= NH; ++m) {
    if (total[m] == 0) continue;  // uniform
    int slot = __shfl(base, m - 1) + below_m[m];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if ((hits >> (4 * (m - 1) + a)) & 1u) {
        if ((unsigned)slot < (unsigned)cap)
          *reinterpret_cast<int4*>(cands + (size_t)(m - 1) * cap + slot) =
              make_int4(m, i, j0 + a, __float_as_int(hk[m][a]));
        ++slot;
      }
    }
  }
}

// Phase 2: work item w = entry * ROWS + row, grid-stride over all items in
// wave-uniform steps so the whole wave reaches the compaction together.
template <int Z, int NH>
__global__ __launch_bounds__(HS_THREADS) void k_harmsum_emit(const float* __restrict__ fop, int64_t ld, int n,
                                                             const int4* __restrict__ hitrows,
                                                             const int32_t* __restrict__ hitrow_count,
                                                             const float* __restrict__ ta,
                                                             fdas_cand* __restrict__ cands, int cap,
                                                             int32_t* __restrict__ counts) {
  constexpr int ROWS = 2 * Z + 1;
  const int64_t items = (int64_t)(*hitrow_count) * ROWS;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * HS_THREADS;
  for (int64_t w0 = (int64_t)blockIdx.x * HS_THREADS + (threadIdx.x & ~63); w0 < items; w0 += stride) {
    const int64_t w = w0 + lane;
    bool act = w < items;
    int4 ent = make_int4(0, 0, 0, 0);
    int r = 0;
    if (act) {
      ent = hitrows[w / ROWS];
      r = (int)(w % ROWS);
      const unsigned word = (unsigned)(r < 32 ? ent.y : (r < 64 ? ent.z : ent.w));
      act = ((word >> (r % 32)) & 1u) != 0;
    }
    if (__ballot(act) == 0ull) continue;  // uniform
    hs_emit_wave<Z, NH>(fop, ld, n, ent.x, r, act, ta, cands, cap, counts, lane);
  }
}

// counts[0 .. nh) = 0 and *extra = 0 in one launch
__global__ void k_fill_counts(int32_t* __restrict__ counts, int nh, int32_t* __restrict__ extra) {
  const int t = threadIdx.x;
  if (t < nh) counts[t] = 0;
  if (extra && t == 63) *extra = 0;
}

// Batch form of phase 2: the entry's trial is in bits 21..31 of its third word.
template <int Z, int NH>
__global__ __launch_bounds__(HS_THREADS) void k_harmsum_emit_batch(const HsTrial* __restrict__ trials,
                                                                   const int4* __restrict__ hitrows,
                                                                   const int32_t* __restrict__ hitrow_count,
                                                                   const float* __restrict__ ta, int cap) {
  constexpr int ROWS = 2 * Z + 1;
  const int64_t items = (int64_t)(*hitrow_count) * ROWS;
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * HS_THREADS;
  // wave-uniform steps; a wave whose active lanes all belong to one trial (the
  // usual case: a phase-1 block appends its entries together) reserves slots
  // per plane for the whole wave, a mixed wave falls back to one atomic per
  // lane and plane
  for (int64_t w0 = (int64_t)blockIdx.x * HS_THREADS + (threadIdx.x & ~63); w0 < items; w0 += stride) {
    const int64_t w = w0 + lane;
    bool act = w < items;
    int4 ent = make_int4(0, 0, 0, 0);
    int r = 0;
    if (act) {
      ent = hitrows[w / ROWS];
      r = (int)(w % ROWS);
      const unsigned w2 = (unsigned)ent.w & 0x1FFFFFu;
      const unsigned word = (unsigned)(r < 32 ? ent.y : (r < 64 ? ent.z : (int)w2));
      act = ((word >> (r % 32)) & 1u) != 0;
    }
    const unsigned long long am = __ballot(act);
    if (am == 0ull) continue;  // uniform
    const int tri = (int)((unsigned)ent.w >> 21);
    const int lead = __builtin_amdgcn_readlane(tri, (int)__builtin_ctzll(am));
    if (__ballot(act && tri != lead) == 0ull) {  // uniform
      const HsTrial& tr = trials[lead];
      hs_emit_wave<Z, NH>(tr.fop, tr.ld, tr.n, ent.x, r, act, ta, tr.cands, cap, tr.counts, lane);
    } else if (act) {
      const HsTrial& tr = trials[tri];
      hs_emit_row<Z, NH>(tr.fop, tr.ld, tr.n, ent.x, r, ta, tr.cands, cap, tr.counts);
    }
  }
}

// counts[0 .. nh) of every trial of a batch set to 0
__global__ void k_zero_counts_batch(const HsTrial* __restrict__ trials, int ntrials, int nh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ntrials * nh) trials[i / nh].counts[i % nh] = 0;
}

__global__ void k_fill_i32(int32_t* p, int count, int32_t value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = value;
}

// Tile order of the 85-row kernel computed on the device (the order
// harmsum_tile_order builds on the host): tile t has the key
// (frac << 6) | (octave + 1), frac = (t - 2^octave) << (top - octave), key 0
// for t = 0; tiles are ranked by key and rank q goes to workgroup
// (q mod per) * 8 + q / per, per = ceil(T / 8).  Keys are distinct, so the
// rank of t is the number of smaller keys.
__device__ __forceinline__ uint64_t tile_key(int t, int top) {
  if (t == 0) return 0;
  const int o = 31 - __clz(t);
  const uint64_t frac = (uint64_t)(t - (1 << o)) << (top - o);
  return (frac << 6) | (uint64_t)(o + 1);
}

__global__ void k_tile_order(int* __restrict__ order, int T, int top, int per) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const uint64_t k = tile_key(t, top);
  int q = 0;
  for (int u = 0; u < T; ++u) q += tile_key(u, top) < k ? 1 : 0;
  order[(q % per) * 8 + q / per] = t;
}

// Scratch of fdas_harmonic_sum_noalloc in static device memory (one copy per
// GPU, kept until the process ends): hit-row counter, tile order, hit-row list.
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 22;
constexpr size_t kNaOrderOff = 256;
constexpr size_t kNaOrderInts = ((size_t)kNoAllocMaxN / (4 * HS_THREADS) + 8 + 63) / 64 * 64;
constexpr size_t kNaHitOff = kNaOrderOff + kNaOrderInts * sizeof(int);
constexpr size_t kNaBytes = kNaHitOff + (size_t)(kNoAllocMaxN / 4) * sizeof(int4);
static __device__ __align__(256) unsigned char scratch[kNaBytes];

}  // namespace

int64_t harmsum_noalloc_max_n() { return kNoAllocMaxN; }
size_t harmsum_noalloc_scratch_bytes() { return kNaBytes; }

hipError_t harmsum_noalloc_scratch(void** ptr) {
  // the caller has made the device current; the address is per device
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t launch_harmsum_noalloc(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm, const float* ta,
                                  fdas_cand* cands, int cap, int32_t* counts, void* scr, int emit_blocks,
                                  int index, hipStream_t s) {
  if (n < 1 || n > kNoAllocMaxN || !scr) return hipErrorInvalidValue;
  unsigned char* base = static_cast<unsigned char*>(scr);
  int* order = reinterpret_cast<int*>(base + kNaOrderOff);
  int4* hitrows = reinterpret_cast<int4*>(base + kNaHitOff);
  int32_t* hit_count = reinterpret_cast<int32_t*>(base);
  const int cols = 4 * HS_THREADS;
  const int T = (int)((n + cols - 1) / cols);
  const int per = (T + 7) / 8;
  const bool ordered = (z_max == 42 && index == FDAS_HSUM_STRETCH) || index == FDAS_HSUM_FUNDAMENTAL ||
                       index == FDAS_HSUM_HIGHEST;
  if (ordered) {
    int top = 0;
    while ((1LL << (top + 1)) <= (int64_t)(T > 2 ? T - 1 : 1)) ++top;
    hipError_t e = launch_fill_i32(order, per * 8, -1, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tile_order, dim3((T + 255) / 256), dim3(256), 0, s, order, T, top, per);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  const HsWork wk{order, per * 8, hitrows, hit_count, emit_blocks};
  return launch_harmsum(fop, n, ld, z_max, n_harm, ta, cands, cap, counts, wk, index, s);
}

int harmsum_tile_columns() { return 4 * HS_THREADS; }

hipError_t launch_fill_i32(int32_t* p, int count, int32_t value, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
  return hipGetLastError();
}

hipError_t launch_zero_counts_batch(const HsTrial* trials, int ntrials, int nh, hipStream_t s) {
  const int total = ntrials * nh;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_counts_batch, dim3((total + 255) / 256), dim3(256), 0, s, trials, ntrials, nh);
  return hipGetLastError();
}

template <int TH>
hipError_t launch_phase1_batch(const HsTrial* trials, int ntrials, int blk_begin, unsigned blocks, int n_harm,
                               const float* ta, int4* hitrows, int32_t* hitrow_count, hipStream_t s) {
  switch (n_harm) {
#define FDAS_HSP_CASE(NH)                                                                                     \
  case NH:                                                                                                    \
    hipLaunchKernelGGL((k_harmsum_z_batch<42, NH, TH>), dim3(blocks), dim3(TH), 0, s, trials, ntrials,        \
                       blk_begin, ta, hitrows, hitrow_count);                                                 \
    break;
    FDAS_HSP_CASE(1)
    FDAS_HSP_CASE(2)
    FDAS_HSP_CASE(3)
    FDAS_HSP_CASE(4)
    FDAS_HSP_CASE(5)
    FDAS_HSP_CASE(6)
    FDAS_HSP_CASE(7)
    FDAS_HSP_CASE(8)
#undef FDAS_HSP_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool harmsum_tile_built(int cols) { return cols == 256 || cols == 512 || cols == 1024; }

hipError_t launch_harmsum_batch85(const HsTrial* trials, int ntrials, int blk_begin, int blk_end, int n_harm,
                                  const float* ta, int cap, int4* hitrows, int32_t* hitrow_count, int eblocks,
                                  int tile_cols, hipStream_t s) {
  if (blk_end <= blk_begin) return hipSuccess;
  hipError_t e = launch_fill_i32(hitrow_count, 1, 0, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)(blk_end - blk_begin);
  switch (tile_cols) {
    case 256: e = launch_phase1_batch<64>(trials, ntrials, blk_begin, blocks, n_harm, ta, hitrows, hitrow_count, s); break;
    case 512: e = launch_phase1_batch<128>(trials, ntrials, blk_begin, blocks, n_harm, ta, hitrows, hitrow_count, s); break;
    case 1024: e = launch_phase1_batch<256>(trials, ntrials, blk_begin, blocks, n_harm, ta, hitrows, hitrow_count, s); break;
    default: return hipErrorInvalidValue;
  }
  if (e != hipSuccess) return e;
  switch (n_harm) {
#define FDAS_HSB_CASE(NH)                                                                                     \
  case NH:                                                                                                    \
    hipLaunchKernelGGL((k_harmsum_emit_batch<42, NH>), dim3(eblocks), dim3(HS_THREADS), 0, s, trials, hitrows, \
                       hitrow_count, ta, cap);                                                                \
    break;
    FDAS_HSB_CASE(1)
    FDAS_HSB_CASE(2)
    FDAS_HSB_CASE(3)
    FDAS_HSB_CASE(4)
    FDAS_HSB_CASE(5)
    FDAS_HSB_CASE(6)
    FDAS_HSB_CASE(7)
    FDAS_HSB_CASE(8)
#undef FDAS_HSB_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_harmsum(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm, const float* ta,
                          fdas_cand* cands, int cap, int32_t* counts, const HsWork& wk, int index, hipStream_t s) {
  // the counts (and the fast path's hit-row counter) start at zero, in one launch
  const bool fast = z_max == 42 && index == FDAS_HSUM_STRETCH;
  hipLaunchKernelGGL(k_fill_counts, dim3(1), dim3(64), 0, s, counts, n_harm, fast ? wk.hitrow_count : nullptr);
  {
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
  }
  if (index == FDAS_HSUM_FUNDAMENTAL || index == FDAS_HSUM_HIGHEST) {
    // column tiles of XT columns, in the order of wk.tile_of_block when given
    const unsigned blocks =
        wk.tile_of_block ? (unsigned)wk.blocks : (unsigned)((n + XT - 1) / XT);
    const int* order = wk.tile_of_block;
    const bool fund = index == FDAS_HSUM_FUNDAMENTAL;
    const bool narrow = 2 * (int64_t)n_harm * n < ((int64_t)1 << 32);  // rho(m j, k) in 32-bit arithmetic
    switch (n_harm) {
#define FDAS_HSX_CASE(NH)                                                                                          \
  case NH:                                                                                                         \
    if (fund)                                                                                                      \
      hipLaunchKernelGGL(k_harmsum_fund<NH>, dim3(blocks), dim3(HS_THREADS), 0, s, fop, ld, (int)n, z_max, order,  \
                         ta, cands, cap, counts);                                                                  \
    else if (narrow)                                                                                               \
      hipLaunchKernelGGL((k_harmsum_high<NH, false>), dim3(blocks), dim3(HS_THREADS), 0, s, fop, ld, (int)n, z_max, \
                         order, ta, cands, cap, counts);                                                           \
    else                                                                                                           \
      hipLaunchKernelGGL((k_harmsum_high<NH, true>), dim3(blocks), dim3(HS_THREADS), 0, s, fop, ld, (int)n, z_max,  \
                         order, ta, cands, cap, counts);                                                           \
    break;
      FDAS_HSX_CASE(1)
      FDAS_HSX_CASE(2)
      FDAS_HSX_CASE(3)
      FDAS_HSX_CASE(4)
      FDAS_HSX_CASE(5)
      FDAS_HSX_CASE(6)
      FDAS_HSX_CASE(7)
      FDAS_HSX_CASE(8)
#undef FDAS_HSX_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int nn = (int)n;
  if (z_max == 42) {
    // two-phase fast path for the 85-template plane
    const unsigned blocks = (unsigned)wk.blocks;
    const unsigned eblocks = (unsigned)(wk.emit_blocks > 0 ? wk.emit_blocks : 1024);
    switch (n_harm) {
#define FDAS_HSZ_CASE(NH)                                                                                          \
  case NH:                                                                                                         \
    hipLaunchKernelGGL((k_harmsum_z<42, NH>), dim3(blocks), dim3(HS_THREADS), 0, s, fop, ld, nn, wk.tile_of_block, \
                       ta, wk.hitrows, wk.hitrow_count);                                                           \
    hipLaunchKernelGGL((k_harmsum_emit<42, NH>), dim3(eblocks), dim3(HS_THREADS), 0, s, fop, ld, nn, wk.hitrows,   \
                       wk.hitrow_count, ta, cands, cap, counts);                                                   \
    break;
      FDAS_HSZ_CASE(1)
      FDAS_HSZ_CASE(2)
      FDAS_HSZ_CASE(3)
      FDAS_HSZ_CASE(4)
      FDAS_HSZ_CASE(5)
      FDAS_HSZ_CASE(6)
      FDAS_HSZ_CASE(7)
      FDAS_HSZ_CASE(8)
#undef FDAS_HSZ_CASE
      default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  const int64_t groups = (n + 3) / 4;
  const unsigned blocks = (unsigned)((groups + HS_THREADS - 1) / HS_THREADS);
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

}  // namespace fdas
