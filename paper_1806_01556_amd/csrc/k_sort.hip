// Canonical ordering of the candidate lists on the device.
//
// The harmonic-sum kernel appends candidates to per-plane lists in arrival
// order.  Algorithm 1 visits cells in (k, i, j) order, so the list is ordered
// by the key ((k-1)*rows + row) * 2^bits_r + r, which is unique per cell.
// The lists are packed into one array and sorted by that key with an LSD
// radix sort (8-bit digits, stable passes):
//   k_sort_hist    per-tile digit histograms (tile = 4096 records)
//   k_sort_scan    exclusive scan of the digit-major histogram table
//   k_sort_scatter stable scatter: ranks within a tile come from wave
//                  ballots (lanes with equal digits) plus per-wave counts
// so the host only copies an already ordered array back.

#include "fdas_internal.h"

namespace fdas {
namespace {

constexpr int ST = 256;            // threads per block
constexpr int SPT = 16;            // records per thread per tile
constexpr int TILE = ST * SPT;     // 4096 records per tile

struct CandKey {
  int rows, z_max, bits_r;
};

__device__ __forceinline__ unsigned long long cand_key(const int4 c, const CandKey kp) {
  const unsigned long long slot = (unsigned long long)((c.x - 1) * kp.rows + (c.y + kp.z_max));
  return (slot << kp.bits_r) | (unsigned long long)(unsigned)c.z;
}

__global__ __launch_bounds__(ST) void k_sort_pack(const int4* __restrict__ planes, int cap, PackPrefix pp,
                                                  int4* __restrict__ out) {
  const int i = blockIdx.x * ST + threadIdx.x;
  if (i >= pp.off[pp.nh]) return;
  int k = 0;
  while (k + 1 < pp.nh && i >= pp.off[k + 1]) ++k;
  out[i] = planes[(size_t)k * cap + (i - pp.off[k])];
}

__global__ __launch_bounds__(ST) void k_sort_hist(const int4* __restrict__ in, int m, int shift, CandKey kp,
                                                  int* __restrict__ hist, int nblk) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * TILE;
#pragma unroll 4
  for (int j = 0; j < SPT; ++j) {
    const int i = base + j * ST + threadIdx.x;
    if (i < m) {
      const int d = (int)((cand_key(in[i], kp) >> shift) & 255ull);
      atomicAdd(&h[d], 1);
    }
  }
  __syncthreads();
  hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of `count` ints in place, one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_sort_scan(int* __restrict__ a, int count) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int per = (count + 1023) / 1024;
  const int lo = min(count, t * per), hi = min(count, lo + per);
  int s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;  // exclusive prefix of this thread's segment
  for (int i = lo; i < hi; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
}

__global__ __launch_bounds__(ST) void k_sort_scatter(const int4* __restrict__ in, int4* __restrict__ out, int m,
                                                     int shift, CandKey kp, const int* __restrict__ offs,
                                                     int nblk) {
  __shared__ int base[256];      // running position per digit inside this tile's output range
  __shared__ int wcnt[ST / 64][256];
  const int t = threadIdx.x;
  const int w = t >> 6;
  base[t] = offs[t * nblk + blockIdx.x];
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

}  // namespace

int sort_tile_count(int m) { return (m + TILE - 1) / TILE; }

hipError_t launch_sort_candidates(const fdas_cand* planes, int cap, const PackPrefix& pp, int rows, int z_max,
                                  int bits_r, fdas_cand* a, fdas_cand* b, int* hist, fdas_cand** sorted,
                                  hipStream_t s) {
  const int m = pp.off[pp.nh];
  *sorted = a;
  if (m == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sort_pack, dim3((m + ST - 1) / ST), dim3(ST), 0, s, reinterpret_cast<const int4*>(planes), cap,
                     pp, reinterpret_cast<int4*>(a));
  const int slot_bits = 32 - __builtin_clz((unsigned)(8 * rows));  // covers (k-1)*rows + row < 8*rows
  const int total_bits = slot_bits + bits_r;
  const int passes = (total_bits + 7) / 8;
  const int nblk = sort_tile_count(m);
  CandKey kp{rows, z_max, bits_r};
  int4* src = reinterpret_cast<int4*>(a);
  int4* dst = reinterpret_cast<int4*>(b);
  for (int p = 0; p < passes; ++p) {
    const int shift = 8 * p;
    hipLaunchKernelGGL(k_sort_hist, dim3(nblk), dim3(ST), 0, s, src, m, shift, kp, hist, nblk);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, hist, 256 * nblk);
    hipLaunchKernelGGL(k_sort_scatter, dim3(nblk), dim3(ST), 0, s, src, dst, m, shift, kp, hist, nblk);
    int4* tmp = src;
    src = dst;
    dst = tmp;
  }
  *sorted = reinterpret_cast<fdas_cand*>(src);
  return hipGetLastError();
}

}  // namespace fdas
