// Canonical ordering of the candidate lists on the device.
//
// The harmonic-sum kernel appends candidates to per-plane lists in arrival
// order.  Algorithm 1 visits cells in (k, i, j) order, so the list is ordered
// by the key ((k-1)*rows + row) * 2^bits_r + r, which is unique per cell.
// The lists are packed into one array and sorted by that key with an LSD
// radix sort (8-bit digits, stable passes):
//   k_sort_pack    packs the per-plane lists (sizes read from the device
//                  counts, so nothing waits for the host) and clears the
//                  per-pass digit totals
//   k_sort_hist    per-tile digit histograms (tile = 1024 records), and the
//                  digit totals of the pass by atomics
//   k_sort_offsets one workgroup per digit turns its row of tile counts into
//                  output offsets (records of smaller digits + the digit's
//                  records in earlier tiles), in place
//   k_sort_scatter stable scatter: ranks within a tile come from wave
//                  ballots (lanes with equal digits) plus per-wave counts
// Every kernel is launched for the largest possible list (n_harm * capacity
// records); tiles past the actual count return at once.
//
// A batch of trials is ordered as one array (k_sort_pack_batch): while they
// are sorted, records carry their trial number in bits 8 and up of the
// harmonic field and the key puts the trial above the plane slot, so the
// sorted array is trial-major with every trial's records in its own canonical
// order; the last scatter pass clears the tag.  The batch record count is
// known to the host, so those launches are sized exactly.

#include <algorithm>

#include "fdas_internal.h"

namespace fdas {
namespace {

constexpr int ST = 256;            // threads per block
constexpr int SPT = 4;             // records per thread per tile
constexpr int TILE = ST * SPT;     // 1024 records per tile

struct CandKey {
  int rows, z_max, bits_r;
  int batch;  // records carry their trial in bits 8.. of the harmonic field
};

__device__ __forceinline__ unsigned long long cand_key(const int4 c, const CandKey kp) {
  const int harm = kp.batch ? (c.x & 255) : c.x;
  unsigned long long slot = (unsigned long long)((harm - 1) * kp.rows + (c.y + kp.z_max));
  if (kp.batch) slot += (unsigned long long)((unsigned)c.x >> 8) * 8ull * (unsigned long long)kp.rows;
  return (slot << kp.bits_r) | (unsigned long long)(unsigned)c.z;
}

// plane offsets of the packed array from the device counts (each plane keeps
// at most cap records, and at most keep of them when keep > 0); returns the total
__device__ __forceinline__ int pack_offsets(const int32_t* __restrict__ counts, int nh, int cap, int (&off)[9],
                                            int keep = 0) {
  off[0] = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int c = k < nh ? min(max(counts[k], 0), cap) : 0;
    if (keep > 0) c = min(c, keep);
    off[k + 1] = off[k] + c;
  }
  return off[8];
}

// records of the list: m_fixed when the host knows it (batch), else from the counts
__device__ __forceinline__ int record_count(const int32_t* __restrict__ counts, int nh, int cap, int m_fixed) {
  if (m_fixed >= 0) return m_fixed;
  int off[9];
  return pack_offsets(counts, nh, cap, off);
}

__global__ __launch_bounds__(ST) void k_sort_pack(const int4* __restrict__ planes, int cap, int nh,
                                                  const int32_t* __restrict__ counts, int4* __restrict__ out,
                                                  int* __restrict__ totals, int ntotals) {
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < ntotals; t += ST) totals[t] = 0;
  int off[9];
  const int m = pack_offsets(counts, nh, cap, off);
  const int i = blockIdx.x * ST + threadIdx.x;
  if (i >= m) return;
  int k = 0;
  while (k + 1 < nh && i >= off[k + 1]) ++k;
  out[i] = planes[(size_t)k * cap + (i - off[k])];
}

__global__ __launch_bounds__(ST) void k_sort_hist(const int4* __restrict__ in, int cap, int nh,
                                                  const int32_t* __restrict__ counts, int m_fixed, int shift,
                                                  CandKey kp, int* __restrict__ hist, int maxblk,
                                                  int* __restrict__ totals) {
  const int m = record_count(counts, nh, cap, m_fixed);
  if ((int)blockIdx.x * TILE >= m) return;  // uniform
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * TILE;
  // one LDS atomic per distinct digit of a wave (lanes with equal digits found
  // by ballots, as in the scatter): skewed digits -- the trial and plane bits
  // of the top passes -- would otherwise serialise 64 atomics on one address
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int i = base + j * ST + threadIdx.x;
    const bool valid = i < m;
    const int d = valid ? (int)((cand_key(in[i], kp) >> shift) & 255ull) : 0;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m1 = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m1 : ~m1;
    }
    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(peers >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)peers, 0u));
    if (valid && rank == 0) atomicAdd(&h[d], __popcll(peers));
  }
  __syncthreads();
  const int v = h[threadIdx.x];
  hist[threadIdx.x * maxblk + blockIdx.x] = v;
  if (v) atomicAdd(&totals[threadIdx.x], v);
}

// Output offsets of the pass: for digit d (workgroup d) and tile b,
// hist[d * maxblk + b] <- (records with a smaller digit) + (records of digit d
// in tiles before b), computed in place by a workgroup-wide scan of the row.
__global__ __launch_bounds__(ST) void k_sort_offsets(int* __restrict__ hist, int maxblk,
                                                     const int* __restrict__ totals, int cap, int nh,
                                                     const int32_t* __restrict__ counts, int m_fixed) {
  const int m = record_count(counts, nh, cap, m_fixed);
  const int nblk = (m + TILE - 1) / TILE;
  if (nblk == 0) return;
  __shared__ int sc[ST];
  __shared__ int s_carry;
  const int d = blockIdx.x, t = threadIdx.x;
  // records whose digit is below d
  sc[t] = t < d ? totals[t] : 0;
  __syncthreads();
  for (int o = ST / 2; o > 0; o >>= 1) {
    if (t < o) sc[t] += sc[t + o];
    __syncthreads();
  }
  if (t == 0) s_carry = sc[0];
  __syncthreads();
  int* row = hist + (size_t)d * maxblk;
  for (int b0 = 0; b0 < nblk; b0 += ST) {
    const int b = b0 + t;
    const int v = b < nblk ? row[b] : 0;
    sc[t] = v;
    __syncthreads();
    for (int o = 1; o < ST; o <<= 1) {
      const int u = t >= o ? sc[t - o] : 0;
      __syncthreads();
      sc[t] += u;
      __syncthreads();
    }
    const int carry = s_carry;
    if (b < nblk) row[b] = carry + sc[t] - v;
    __syncthreads();
    if (t == ST - 1) s_carry = carry + sc[t];
    __syncthreads();
  }
}

__global__ __launch_bounds__(ST) void k_sort_scatter(const int4* __restrict__ in, int4* __restrict__ out, int cap,
                                                     int nh, const int32_t* __restrict__ counts, int m_fixed,
                                                     int shift, CandKey kp, const int* __restrict__ offs, int maxblk,
                                                     int untag) {
  const int m = record_count(counts, nh, cap, m_fixed);
  if ((int)blockIdx.x * TILE >= m) return;  // uniform
  __shared__ int base[256];      // running position per digit inside this tile's output range
  __shared__ int wcnt[ST / 64][256];
  const int t = threadIdx.x;
  const int w = t >> 6;
  base[t] = offs[(size_t)t * maxblk + blockIdx.x];
#pragma unroll
  for (int q = 0; q < ST / 64; ++q) wcnt[q][t] = 0;
  __syncthreads();
  const int tile0 = blockIdx.x * TILE;
  for (int j = 0; j < SPT; ++j) {
    const int i = tile0 + j * ST + t;
    const bool valid = i < m;
    int4 rec = make_int4(0, 0, 0, 0);
    int d = 0;
    if (valid) {
      rec = in[i];
      d = (int)((cand_key(rec, kp) >> shift) & 255ull);
    }
    // lanes of this wave holding the same digit
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const unsigned long long m1 = __ballot((d >> b) & 1);
      peers &= ((d >> b) & 1) ? m1 : ~m1;
    }
    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(peers >> 32),
                                               __builtin_amdgcn_mbcnt_lo((unsigned)peers, 0u));
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      if (untag) rec.x &= 255;
      out[pos] = rec;
    }
    __syncthreads();
    // advance the running bases and clear the per-wave counts
    {
      int add = 0;
#pragma unroll
      for (int q = 0; q < ST / 64; ++q) {
        add += wcnt[q][t];
        wcnt[q][t] = 0;
      }
      base[t] += add;
    }
    __syncthreads();
  }
}

// out[t * nh + k] = ptrs[t][k]: the counts of every trial of a batch in one array
__global__ void k_gather_counts(int32_t* const* __restrict__ ptrs, int count, int nh, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count * nh) out[i] = ptrs[i / nh][i % nh];
}

// Batch pack: record i of the packed array belongs to the last trial whose
// first record is <= i (empty trials share their successor's offset), then to
// that trial's plane by its clamped counts.  The trial is tagged into the
// harmonic field.  Block 0 also clears the per-pass digit totals.
__global__ __launch_bounds__(ST) void k_sort_pack_batch(const RbTrial* __restrict__ tr, int count, int cap, int nh,
                                                        int m, int4* __restrict__ out, int* __restrict__ totals,
                                                        int ntotals) {
  if (blockIdx.x == 0)
    for (int t = threadIdx.x; t < ntotals; t += ST) totals[t] = 0;
  const int i = blockIdx.x * ST + threadIdx.x;
  if (i >= m) return;
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tr[mid].off <= (int64_t)i) lo = mid; else hi = mid - 1;
  }
  int off[9];
  pack_offsets(tr[lo].counts, nh, cap, off);
  const int j = i - (int)tr[lo].off;
  int k = 0;
  while (k + 1 < nh && j >= off[k + 1]) ++k;
  int4 rec = tr[lo].cands[(size_t)k * cap + (j - off[k])];
  rec.x |= lo << 8;
  out[i] = rec;
}

// Top-k selection of Table 1's N_cand per plane, on the ordered array: block
// k keeps the top_k highest powers of plane k (ties: lower z, then lower r --
// the earlier record of the (z, r)-ordered plane) and writes them, still in
// (z, r) order, after the kept records of the planes before it.  The k-th
// largest of the distinct keys (power bits << 32 | ~position) is found by an
// 8-bit radix select from the top digit; the records with a key at least as
// large are compacted in order by a workgroup scan.
constexpr int TK = 1024;  // threads of the selection

__device__ __forceinline__ unsigned long long topk_key(const int4* __restrict__ plane, int p) {
  // powers of candidates are above a positive threshold: their bits order them
  return ((unsigned long long)(unsigned)plane[p].w << 32) | (unsigned long long)(~(unsigned)p);
}

__global__ __launch_bounds__(TK) void k_topk(const int4* __restrict__ sorted, int cap, int nh,
                                             const int32_t* __restrict__ counts, int top_k,
                                             int4* __restrict__ out) {
  __shared__ int s_hist[256];
  __shared__ int s_scan[TK];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_need;
  const int k = blockIdx.x, t = threadIdx.x;
  if (k >= nh) return;
  int off[9], okeep[9];
  pack_offsets(counts, nh, cap, off);
  pack_offsets(counts, nh, cap, okeep, top_k);
  const int m = off[k + 1] - off[k];
  const int4* plane = sorted + off[k];
  int4* dst = out + okeep[k];
  if (m <= top_k) {
    for (int i = t; i < m; i += TK) dst[i] = plane[i];
    return;
  }
  // radix select of the top_k-th largest key
  if (t == 0) {
    s_prefix = 0ull;
    s_need = top_k;
  }
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int d = t; d < 256; d += TK) s_hist[d] = 0;
    __syncthreads();
    const unsigned long long prefix = s_prefix;
    const unsigned long long hmask = shift == 56 ? 0ull : (~0ull << (shift + 8));
    for (int i = t; i < m; i += TK) {
      const unsigned long long key = topk_key(plane, i);
      if ((key & hmask) == prefix) atomicAdd(&s_hist[(int)((key >> shift) & 255ull)], 1);
    }
    __syncthreads();
    if (t == 0) {
      // the digit D at which the count of keys with a larger digit stays
      // below the need and the count with digit >= D reaches it
      int need = s_need, above = 0, D = 255;
      for (; D > 0; --D) {
        if (above + s_hist[D] >= need) break;
        above += s_hist[D];
      }
      s_need = need - above;
      s_prefix = prefix | ((unsigned long long)D << shift);
    }
    __syncthreads();
  }
  const unsigned long long kth = s_prefix;  // keys are distinct: exactly top_k are >= kth
  // stable compaction of the keys >= kth
  int base = 0;
  for (int i0 = 0; i0 < m; i0 += TK) {
    const int i = i0 + t;
    const int f = (i < m && topk_key(plane, i) >= kth) ? 1 : 0;
    s_scan[t] = f;
    __syncthreads();
    for (int o = 1; o < TK; o <<= 1) {
      const int u = t >= o ? s_scan[t - o] : 0;
      __syncthreads();
      s_scan[t] += u;
      __syncthreads();
    }
    if (f) dst[base + s_scan[t] - 1] = plane[i];
    base += s_scan[TK - 1];
    __syncthreads();
  }
}

// The ordered records and the counts written straight into page-locked host
// memory (device-visible pointers), so the host waits once: records
// [0, min(total, out_cap)) of `sorted` (each plane limited to keep records
// when keep > 0: `sorted` is then the top-k output), counts[0 .. nh).
__global__ __launch_bounds__(ST) void k_copy_out(const int4* __restrict__ sorted, int cap, int nh,
                                                 const int32_t* __restrict__ counts, int out_cap, int keep,
                                                 int4* __restrict__ out, int32_t* __restrict__ counts_out) {
  int off[9];
  const int m = min(pack_offsets(counts, nh, cap, off, keep), out_cap);
  if (blockIdx.x == 0 && (int)threadIdx.x < nh) counts_out[threadIdx.x] = counts[threadIdx.x];
  for (int i = blockIdx.x * ST + threadIdx.x; i < m; i += gridDim.x * ST) out[i] = sorted[i];
}

}  // namespace

hipError_t launch_copy_out(const fdas_cand* sorted, int cap, int nh, const int32_t* counts, int out_cap,
                           fdas_cand* out, int32_t* counts_out, hipStream_t s, int keep) {
  const int blocks = std::max(1, std::min(1024, (nh * cap + ST - 1) / ST));
  hipLaunchKernelGGL(k_copy_out, dim3(blocks), dim3(ST), 0, s, reinterpret_cast<const int4*>(sorted), cap, nh,
                     counts, out_cap, keep, reinterpret_cast<int4*>(out), counts_out);
  return hipGetLastError();
}

hipError_t launch_topk(const fdas_cand* sorted, int cap, int nh, const int32_t* counts, int top_k, fdas_cand* out,
                       hipStream_t s) {
  if (top_k <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_topk, dim3(nh), dim3(TK), 0, s, reinterpret_cast<const int4*>(sorted), cap, nh, counts, top_k,
                     reinterpret_cast<int4*>(out));
  return hipGetLastError();
}

hipError_t launch_gather_counts(int32_t* const* ptrs, int count, int nh, int32_t* out, hipStream_t s) {
  const int total = count * nh;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_counts, dim3((total + 255) / 256), dim3(256), 0, s, ptrs, count, nh, out);
  return hipGetLastError();
}

int sort_tile_count(int m) { return (m + TILE - 1) / TILE; }

int sort_passes(int rows, int bits_r) {
  const int slot_bits = 32 - __builtin_clz((unsigned)(8 * rows));  // covers (k-1)*rows + row < 8*rows
  return (slot_bits + bits_r + 7) / 8;
}

hipError_t launch_sort_candidates(const fdas_cand* planes, int cap, int nh, const int32_t* counts, int rows,
                                  int z_max, int bits_r, fdas_cand* a, fdas_cand* b, int* hist, int* totals,
                                  fdas_cand** sorted, hipStream_t s) {
  const int maxm = nh * cap;
  const int maxblk = sort_tile_count(maxm);
  const int passes = sort_passes(rows, bits_r);
  hipLaunchKernelGGL(k_sort_pack, dim3((maxm + ST - 1) / ST), dim3(ST), 0, s, reinterpret_cast<const int4*>(planes),
                     cap, nh, counts, reinterpret_cast<int4*>(a), totals, 256 * passes);
  CandKey kp{rows, z_max, bits_r, 0};
  int4* src = reinterpret_cast<int4*>(a);
  int4* dst = reinterpret_cast<int4*>(b);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    int* tot = totals + 256 * p;
    hipLaunchKernelGGL(k_sort_hist, dim3(maxblk), dim3(ST), 0, s, src, cap, nh, counts, -1, shift, kp, hist, maxblk,
                       tot);
    hipLaunchKernelGGL(k_sort_offsets, dim3(256), dim3(ST), 0, s, hist, maxblk, tot, cap, nh, counts, -1);
    hipLaunchKernelGGL(k_sort_scatter, dim3(maxblk), dim3(ST), 0, s, src, dst, cap, nh, counts, -1, shift, kp, hist,
                       maxblk, 0);
    int4* tmp = src;
    src = dst;
    dst = tmp;
  }
  *sorted = reinterpret_cast<fdas_cand*>(src);
  return hipGetLastError();
}

int sort_passes_batch(int count, int rows, int bits_r) {
  const int slot_bits = 32 - __builtin_clz((unsigned)(8 * rows * count));  // trial * 8 * rows + plane slot
  return (slot_bits + bits_r + 7) / 8;
}

hipError_t launch_sort_batch(const RbTrial* tab, int count, int cap, int nh, int m, int rows, int z_max, int bits_r,
                             fdas_cand* a, fdas_cand* b, int* hist, int* totals, fdas_cand** sorted, hipStream_t s) {
  *sorted = a;
  if (m <= 0) return hipSuccess;
  const int nblk = sort_tile_count(m);
  const int passes = sort_passes_batch(count, rows, bits_r);
  hipLaunchKernelGGL(k_sort_pack_batch, dim3((m + ST - 1) / ST), dim3(ST), 0, s, tab, count, cap, nh, m,
                     reinterpret_cast<int4*>(a), totals, 256 * passes);
  CandKey kp{rows, z_max, bits_r, 1};
  int4* src = reinterpret_cast<int4*>(a);
  int4* dst = reinterpret_cast<int4*>(b);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    int* tot = totals + 256 * p;
    hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(ST), 0, s, src, cap, nh, nullptr, m, shift, kp, hist, nblk, tot);
    hipLaunchKernelGGL(k_sort_offsets, dim3(256), dim3(ST), 0, s, hist, nblk, tot, cap, nh, nullptr, m);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(ST), 0, s, src, dst, cap, nh, nullptr, m, shift, kp, hist,
                       nblk, p == passes - 1 ? 1 : 0);
    int4* tmp = src;
    src = dst;
    dst = tmp;
  }
  *sorted = reinterpret_cast<fdas_cand*>(src);
  return hipGetLastError();
}

}  // namespace fdas
