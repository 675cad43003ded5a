// Host-side FP64 arithmetic of plan creation: acceleration templates, their
// overlap-save spectra, FFT twiddle tables and detection thresholds.
//
// Templates.  FDAS correlates the spectrum with the conjugate Fourier response
// of a signal whose frequency drifts by z bins over the observation (the paper
// names the Ransom et al. correlation technique and gives 85 filters of up to
// ~400 taps, Section 1 and Table 1, but prints no coefficients).  Here
//   A(q, z) = integral_0^1 exp(i*pi*(z*u^2 + (2q - z)*u)) du,
// evaluated by composite Gauss-Legendre quadrature (nodes from Newton's method
// on the Legendre recurrence), and
//   h_z[d] = conj(A(-d, z)) / sqrt(E_z),  E_z = sum_d |A(-d, z)|^2,
//   d in [-L/2, L/2 - 1],  L(z) = 2*(8 + ceil(4.5*|z|)).
// The integrand's phase turns at most pi*(|z| + 2|q|) radians per unit u; the
// panel count keeps that below ~5.4 rad per 16-node panel, where the
// Gauss-Legendre remainder is far below double rounding.
//
// Thresholds.  HP_k of unit-mean exponential noise is Gamma(k, 1); its survival
// function for integer k is exp(-T) * sum_{n<k} T^n / n!.  T_k solves
// survival = p_fa (bisection, then Newton on the logarithm).

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "fdas_internal.h"

namespace fdas {

using cd = std::complex<double>;

int tap_count(int z) {
  const int az = z < 0 ? -z : z;
  return 2 * (8 + (9 * az + 1) / 2);
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = M_PI;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double r = std::cos(pi * (i + 0.75) / (n + 0.5));
    double dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      // p1 = P_n(r), p0 = P_{n-1}(r)
      dp = n * (r * p1 - p0) / (r * r - 1.0);
      const double dr = p1 / dp;
      r -= dr;
      if (std::fabs(dr) < 1e-16) break;
    }
    // recompute the derivative at the converged root
    double p0 = 1.0, p1 = r;
    for (int k = 2; k <= n; ++k) {
      const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (r * p1 - p0) / (r * r - 1.0);
    x[i] = -r;
    x[n - 1 - i] = r;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - r * r) * dp * dp);
  }
}

// exp(2*pi*i*t) for a real t, with t reduced to [0, 1) first.
static inline cd expi2pi(double t) {
  t -= std::floor(t);
  const double a = 2.0 * M_PI * t;
  return cd(std::cos(a), std::sin(a));
}

void template_taps(int z, std::vector<cd>& h) {
  const int L = tap_count(z);
  const int half = L / 2;
  // taps need A(q, z) for q = -d, d in [-half, half-1]  ->  q in [1-half, half]
  const int q_lo = 1 - half, q_hi = half;
  const double max_rate = M_PI * (std::fabs((double)z) + 2.0 * std::max(std::abs(q_lo), std::abs(q_hi)));
  const int order = 16;
  int panels = (int)std::ceil(max_rate / 5.0);
  panels = std::max(panels, 16);
  std::vector<double> gx, gw;
  gauss_legendre(order, gx, gw);
  const int nn = panels * order;
  std::vector<double> u(nn);
  std::vector<cd> g(nn), step(nn), cur(nn);
  for (int p = 0; p < panels; ++p) {
    const double a = (double)p / panels, b = (double)(p + 1) / panels;
    for (int m = 0; m < order; ++m) {
      const double uu = 0.5 * (b - a) * gx[m] + 0.5 * (a + b);
      const double ww = 0.5 * (b - a) * gw[m];
      const int idx = p * order + m;
      u[idx] = uu;
      // exp(i*pi*z*(u^2 - u)) carries the drift; exp(2*pi*i*q*u) the offset.
      g[idx] = ww * expi2pi(0.5 * z * (uu * uu - uu));
      step[idx] = expi2pi(uu);
    }
  }
  std::vector<cd> A(q_hi - q_lo + 1);
  for (int q = q_lo; q <= q_hi; ++q) {
    const int k = q - q_lo;
    if (k % 32 == 0) {
      for (int m = 0; m < nn; ++m) cur[m] = expi2pi((double)q * u[m]);
    }
    cd acc(0.0, 0.0);
    for (int m = 0; m < nn; ++m) {
      acc += g[m] * cur[m];
      cur[m] *= step[m];
    }
    A[k] = acc;
  }
  double energy = 0.0;
  for (const cd& a : A) energy += std::norm(a);
  const double inv = 1.0 / std::sqrt(energy);
  h.assign(L, cd(0.0, 0.0));
  for (int t = 0; t < L; ++t) {
    const int d = t - half;
    const int q = -d;
    h[t] = std::conj(A[q - q_lo]) * inv;
  }
}

void template_bank(int z_max, std::vector<std::vector<cd>>& bank) {
  const int rows = 2 * z_max + 1;
  bank.assign(rows, {});
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned w = 0; w < hw; ++w) {
    th.emplace_back([&, w]() {
      for (int r = (int)w; r < rows; r += (int)hw) template_taps(r - z_max, bank[r]);
    });
  }
  for (auto& t : th) t.join();
}

void ols_spectra(const std::vector<std::vector<cd>>& bank, int C, int P, std::vector<float>& out) {
  // g[t] = h[t - P] on t in [P - L/2, P + L/2 - 1];  H[k] = (1/C) sum_t g[t] e^{+2 pi i t k / C}.
  const int rows = (int)bank.size();
  out.assign((size_t)rows * C * 2, 0.0f);
  std::vector<cd> tw(C);
  for (int m = 0; m < C; ++m) tw[m] = expi2pi((double)m / C);
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> th;
  for (unsigned w = 0; w < hw; ++w) {
    th.emplace_back([&, w]() {
      for (int r = (int)w; r < rows; r += (int)hw) {
        const std::vector<cd>& h = bank[r];
        const int L = (int)h.size();
        const int t0 = P - L / 2;
        for (int k = 0; k < C; ++k) {
          cd acc(0.0, 0.0);
          for (int s = 0; s < L; ++s) {
            const long long t = t0 + s;
            acc += h[s] * tw[(size_t)((t * k) % C)];
          }
          acc /= (double)C;
          out[((size_t)r * C + k) * 2 + 0] = (float)acc.real();
          out[((size_t)r * C + k) * 2 + 1] = (float)acc.imag();
        }
      }
    });
  }
  for (auto& t : th) t.join();
}

void direct_pack(const std::vector<std::vector<cd>>& bank, int z_max, std::vector<float>& Bpk,
                 std::vector<int>& tiles, std::vector<int>& rows, int* P_max, int* P8_max) {
  // member order by |z|: 0, -1, 1, -2, 2, ...
  std::vector<int> order;
  order.push_back(0);
  for (int a = 1; a <= z_max; ++a) {
    order.push_back(-a);
    order.push_back(a);
  }
  const int T = ((int)order.size() + 7) / 8;
  tiles.assign((size_t)T * 4, 0);
  rows.assign((size_t)T * 8, -1);
  Bpk.clear();
  int pairs = 0, pm = 0, p8m = 0;
  for (int g = 0; g < T; ++g) {
    const int cnt = std::min(8, (int)order.size() - 8 * g);
    int P = 0;
    for (int t = 0; t < cnt; ++t) P = std::max(P, tap_count(order[8 * g + t]) / 2);
    const int P8 = (P + 7) / 8 * 8;  // pairs padded with zero values to a multiple of 8
    pm = std::max(pm, P);
    p8m = std::max(p8m, P8);
    tiles[4 * g + 0] = P;
    tiles[4 * g + 1] = pairs;
    tiles[4 * g + 2] = cnt;
    tiles[4 * g + 3] = P8;
    for (int t = 0; t < cnt; ++t) rows[8 * g + t] = order[8 * g + t] + z_max;
    for (int p = 0; p < P8; ++p) {
      for (int lane = 0; lane < 64; ++lane) {
        const int col = lane & 15, k = lane >> 4;
        const int slot = col >> 1, part = col & 1;
        const int d = -P + 2 * p + (k >> 1);  // tap of this k
        cd h(0.0, 0.0);
        if (slot < cnt && p < P) {
          const int z = order[8 * g + slot];
          const std::vector<cd>& hz = bank[z + z_max];
          const int L = (int)hz.size();
          const int t = d + L / 2;
          if (t >= 0 && t < L) h = hz[t];
        }
        // (Re X, Im X) against the Re-column: (Re h, -Im h); against the Im-column: (Im h, Re h)
        const bool im_x = (k & 1) != 0;
        const double v = part == 0 ? (im_x ? -h.imag() : h.real()) : (im_x ? h.real() : h.imag());
        Bpk.push_back((float)v);
      }
    }
    pairs += P8;
  }
  *P_max = pm;
  *P8_max = p8m;
}

namespace {

// IEEE binary16 and bfloat16 bit patterns, round to nearest even
uint16_t to_f16_bits(float v) { return __builtin_bit_cast(uint16_t, (_Float16)v); }
float from_f16_bits(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
uint16_t to_bf16_bits(float v) {
  uint32_t u = __builtin_bit_cast(uint32_t, v);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // NaN stays NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float from_bf16_bits(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

}  // namespace

void direct_pack_split(const std::vector<std::vector<cd>>& bank, int z_max, bool bf16, std::vector<uint16_t>& Bsp,
                       std::vector<float>& tscale, std::vector<int>& tiles, std::vector<int>& rows, int* P_max,
                       int* P8_max) {
  std::vector<float> Bpk;
  direct_pack(bank, z_max, Bpk, tiles, rows, P_max, P8_max);  // same order, tiles and supports
  const int T = (int)tiles.size() / 4;
  tscale.assign(T, 1.0f);
  Bsp.clear();
  int groups = 0;
  for (int g = 0; g < T; ++g) {
    const int P = tiles[4 * g + 0], first_pair = tiles[4 * g + 1], P8 = tiles[4 * g + 3];
    // FP32 value of (tap d, part) for column col, read back from the FP32 pack:
    // pair p holds taps -P + 2p (k = 0, 1) and -P + 2p + 1 (k = 2, 3)
    auto val = [&](int d, int part, int col) -> float {
      const int t = d + P;
      const int p = t >> 1, k = 2 * (t & 1) + part;
      if (p >= P8) return 0.0f;
      return Bpk[((size_t)(first_pair + p)) * 64 + k * 16 + col];
    };
    float mx = 0.0f;
    for (int p = 0; p < P8 * 64; ++p) mx = std::max(mx, std::fabs(Bpk[(size_t)first_pair * 64 + p]));
    const int eh = mx > 0.0f ? 14 - std::ilogb(mx) : 0;
    tscale[g] = std::ldexp(1.0f, -eh);
    tiles[4 * g + 1] = groups;
    const int G16 = P8 / 8;
    for (int q = 0; q < G16; ++q) {
      uint16_t hi[64 * 8], lo[64 * 8];
      for (int lane = 0; lane < 64; ++lane) {
        const int col = lane & 15, kg = lane >> 4;
        for (int e = 0; e < 8; ++e) {
          const int d = -P + 16 * q + 4 * kg + e / 2;
          const float v = std::ldexp(val(d, e & 1, col), eh);
          uint16_t h, l;
          if (bf16) {
            h = to_bf16_bits(v);
            l = to_bf16_bits(v - from_bf16_bits(h));
          } else {
            h = to_f16_bits(v);
            l = to_f16_bits(v - from_f16_bits(h));
          }
          hi[lane * 8 + e] = h;
          lo[lane * 8 + e] = l;
        }
      }
      Bsp.insert(Bsp.end(), hi, hi + 64 * 8);
      Bsp.insert(Bsp.end(), lo, lo + 64 * 8);
    }
    groups += G16;
  }
}

void fft_twiddles(int C, std::vector<float>& tw1, std::vector<float>& tw2) {
  // tw1[nb][t] = e^{+2 pi i nb t / C} (nb < 16, t < C/16);
  // tw2[q][c] = e^{+2 pi i q c / M} (q < 16, c < M/16, M = C/16);
  // tw2[16][p] = e^{+2 pi i p / 32} (p < 16; used by the 8192-point transform)
  const int NT = C / 16, M = C / 16, TW2 = M / 16;
  tw1.assign((size_t)16 * NT * 2, 0.0f);
  tw2.assign((size_t)17 * TW2 * 2, 0.0f);
  for (int nb = 0; nb < 16; ++nb)
    for (int t = 0; t < NT; ++t) {
      const cd w = expi2pi((double)((long long)nb * t % C) / C);
      tw1[((size_t)nb * NT + t) * 2 + 0] = (float)w.real();
      tw1[((size_t)nb * NT + t) * 2 + 1] = (float)w.imag();
    }
  for (int q = 0; q < 16; ++q)
    for (int c = 0; c < TW2; ++c) {
      const cd w = expi2pi((double)(q * c % M) / M);
      tw2[((size_t)q * TW2 + c) * 2 + 0] = (float)w.real();
      tw2[((size_t)q * TW2 + c) * 2 + 1] = (float)w.imag();
    }
  for (int p = 0; p < 16 && p < TW2; ++p) {
    const cd w = expi2pi((double)p / 32.0);
    tw2[((size_t)16 * TW2 + p) * 2 + 0] = (float)w.real();
    tw2[((size_t)16 * TW2 + p) * 2 + 1] = (float)w.imag();
  }
}

static double log_survival(int k, double t) {
  double term = 1.0, acc = 1.0;
  for (int n = 1; n < k; ++n) {
    term *= t / n;
    acc += term;
  }
  return -t + std::log(acc);
}

double erlang_threshold(int k, double p_fa) {
  const double target = std::log(p_fa);
  double lo = 0.0, hi = 1.0;
  while (log_survival(k, hi) > target) hi *= 2.0;
  for (int it = 0; it < 200 && hi - lo > 1e-13 * hi; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (log_survival(k, mid) > target) lo = mid; else hi = mid;
  }
  double t = 0.5 * (lo + hi);
  for (int it = 0; it < 4; ++it) {
    // d/dt log S = -(t^{k-1}/(k-1)!) / sum_{n<k} t^n/n!
    double term = 1.0, acc = 1.0;
    for (int n = 1; n < k; ++n) {
      term *= t / n;
      acc += term;
    }
    const double dlog = -term / acc;
    const double f = log_survival(k, t) - target;
    t -= f / dlog;
  }
  return t;
}

void stretch_source_rows(int Z, int nh, int* lo, int* hi) {
  // source row of row r for harmonic k: trunc((r - Z) / k) + Z (C division)
  *lo = 0;
  *hi = -1;
  for (int k = 2; k <= nh; ++k) {
    const int a = (0 - Z) / k + Z, b = (2 * Z - Z) / k + Z;
    if (*hi < *lo) {
      *lo = a;
      *hi = b;
    } else {
      *lo = std::min(*lo, a);
      *hi = std::max(*hi, b);
    }
  }
}

// Tile order of the harmonic-sum kernel.  The stretched reads of tile t come
// from tiles t/k; for k = 2, 4, 8 these are the doubling chain below t.  Tiles
// are sorted by the fraction of log2(t) (the bits after the leading one,
// left-aligned) and then by octave, which puts every chain t, 2t(+1), 4t(+3),
// 8t(+7) next to each other, so a tile's k = 2, 4, 8 sources were read moments
// before.  The sorted list is split into 8 contiguous segments, one per XCD
// (workgroup b runs on XCD b mod 8), so a chain also shares one L2.
void harmsum_tile_order(int64_t n, std::vector<int>& tile_of_block, int cols) {
  const int T = (int)((n + cols - 1) / cols);
  int top = 0;
  while ((1LL << (top + 1)) <= (int64_t)std::max(1, T - 1)) ++top;  // octave of the largest tile index
  std::vector<std::pair<uint64_t, int>> key(T);
  for (int t = 0; t < T; ++t) {
    if (t == 0) {
      key[t] = {0, t};
      continue;
    }
    int o = 0;
    while ((1LL << (o + 1)) <= t) ++o;
    const uint64_t frac = (uint64_t)(t - (1LL << o)) << (top - o);
    key[t] = {(frac << 6) | (uint64_t)(o + 1), t};
  }
  std::sort(key.begin(), key.end());
  const int xcd = 8;
  const int per = (T + xcd - 1) / xcd;
  tile_of_block.assign((size_t)per * xcd, -1);
  for (int b = 0; b < per * xcd; ++b) {
    const int seg = b % xcd, q = b / xcd;
    const int idx = seg * per + q;
    if (q < per && idx < T) tile_of_block[b] = key[idx].second;
  }
}

}  // namespace fdas
