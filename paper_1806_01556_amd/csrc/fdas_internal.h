// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/fdas.h"

namespace fdas {

// ---- FP64 plan arithmetic (fdas_math.cpp) ---------------------------------
int tap_count(int z);
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void template_taps(int z, std::vector<std::complex<double>>& h);
void template_bank(int z_max, std::vector<std::vector<std::complex<double>>>& bank);
void ols_spectra(const std::vector<std::vector<std::complex<double>>>& bank, int C, int P,
                 std::vector<float>& out);
void fft_twiddles(std::vector<float>& tw1, std::vector<float>& tw2);
double erlang_threshold(int k, double p_fa);

// ---- overlap-save geometry -------------------------------------------------
constexpr int kOlsC = 4096;      // FFT length of one chunk
constexpr int kOlsThreads = 256; // threads per workgroup (16 points each)

struct OlsGeom {
  int C;   // chunk FFT length
  int P;   // left context = max L/2
  int V;   // valid outputs per chunk = C - (L_max - 1)
};

// ---- kernel launchers (k_*.hip) -------------------------------------------
hipError_t launch_ols_conv(const float2* x, int64_t n, float* fop, int64_t ld,
                           const float2* H, const float2* tw1, const float2* tw2,
                           int rows, int tpg, const OlsGeom& g, hipStream_t s);

hipError_t launch_harmsum(const float* fop, int64_t n, int64_t ld, int z_max, int n_harm,
                          const float* ta, fdas_cand* cands, int cap, int32_t* counts,
                          hipStream_t s);

hipError_t launch_fill_i32(int32_t* p, int count, int32_t value, hipStream_t s);

}  // namespace fdas
