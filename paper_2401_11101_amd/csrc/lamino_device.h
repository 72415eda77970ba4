// Device helpers shared by the kernel sources: typed loads and stores of
// data / spectra, and the in-place block FFT over LDS.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lamino_common.h"
#include "lamino_internal.h"

namespace lam {

constexpr int NTF = 512;       // threads per block of the FFT kernels
constexpr int LDS_CPLX = 4096; // complex values per FFT block (one 32 KB buffer)
constexpr int FFT_IO = LDS_CPLX / NTF;  // loads in flight per thread when staging a block

// ------------------------------------------------------------ load/store
__device__ __forceinline__ float2 ld_c(const void* p, size_t i, int dt) {
  if (dt == LAMINO_F32) return reinterpret_cast<const float2*>(p)[i];
  if (dt == LAMINO_F16) return __half22float2(reinterpret_cast<const __half2*>(p)[i]);
  return __bfloat1622float2(reinterpret_cast<const __hip_bfloat162*>(p)[i]);
}
__device__ __forceinline__ void st_c(void* p, size_t i, float2 v, int dt) {
  if (dt == LAMINO_F32) reinterpret_cast<float2*>(p)[i] = v;
  else if (dt == LAMINO_F16) reinterpret_cast<__half2*>(p)[i] = __float22half2_rn(v);
  else reinterpret_cast<__hip_bfloat162*>(p)[i] = __float22bfloat162_rn(v);
}
__device__ __forceinline__ float ld_r(const void* p, size_t i, int dt) {
  if (dt == LAMINO_F32) return reinterpret_cast<const float*>(p)[i];
  if (dt == LAMINO_U8) return (float)reinterpret_cast<const unsigned char*>(p)[i];
  if (dt == LAMINO_U16) return (float)reinterpret_cast<const unsigned short*>(p)[i];
  if (dt == LAMINO_F16) return __half2float(reinterpret_cast<const __half*>(p)[i]);
  return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(p)[i]);
}
__device__ __forceinline__ void st_r(void* p, size_t i, float v, int dt) {
  if (dt == LAMINO_F32) reinterpret_cast<float*>(p)[i] = v;
  else if (dt == LAMINO_F16) reinterpret_cast<__half*>(p)[i] = __float2half_rn(v);
  else reinterpret_cast<__hip_bfloat16*>(p)[i] = __float2bfloat16(v);
}

// Line integral from raw counts (recording model raw = exp(-d)(flat - dark)
// + dark): -log of the flat/dark-corrected ratio, clamped below at min_ratio;
// a pixel with flat <= dark takes min_ratio.
__device__ __forceinline__ float flat_dark_log(float raw, float dark, float flat, float min_ratio) {
  const float den = flat - dark;
  const float ratio = den > 0.f ? (raw - dark) / den : min_ratio;
  return -logf(fmaxf(ratio, min_ratio));
}

// ------------------------------------------------------------ block FFT
// One Stockham pass of radix R over B transforms of length N = 2^log2N in
// place: each thread reads one butterfly's inputs, twiddles and transforms
// them in registers, and writes the outputs after a barrier.  N / R <= NTF,
// so a round covers NTF R / N whole transforms.
template <int R>
__device__ __forceinline__ void fft_pass_inplace(float2* a, int log2N, int B, int log2Ns,
                                                 const float2* __restrict__ tw, int log2max,
                                                 bool inv) {
  constexpr int LR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int N = 1 << log2N;
  const int lper = log2N - LR;
  const int per = 1 << lper;
  const int tb = per >= NTF ? 1 : NTF >> lper;  // transforms per round
  const int t = threadIdx.x;
  const int j = t & (per - 1);
  for (int b0 = 0; b0 < B; b0 += tb) {
    const int bb = b0 + (t >> lper);
    const bool act = t < tb * per && bb < B;
    float2 v[R];
    if (act) {
      if constexpr (R == 8) {
        r8_load(a + bb * N, N, j, v);
        r8_compute(j, log2Ns, tw, log2max, inv, v);
      } else if constexpr (R == 4) {
        r4_load(a + bb * N, N, j, v);
        r4_compute(j, log2Ns, tw, log2max, inv, v);
      } else {
        r2_load(a + bb * N, N, j, v);
        r2_compute(j, log2Ns, tw, log2max, inv, v);
      }
    }
    __syncthreads();
    if (act) rstore<R>(a + bb * N, j, log2Ns, v);
    __syncthreads();
  }
}

// B transforms of length 2^log2N stored back to back in LDS at `a`
// (B * N <= LDS_CPLX, N <= 4096), transformed in place.
__device__ inline void block_fft(float2* a, int log2N, int B, const float2* __restrict__ tw, int log2max,
                          bool inv) {
  const int np = fft_num_passes(log2N);
  for (int p = 0; p < np; ++p) {
    const FftPass f = fft_pass(log2N, p);
    if (f.radix == 8) fft_pass_inplace<8>(a, log2N, B, f.log2Ns, tw, log2max, inv);
    else if (f.radix == 4) fft_pass_inplace<4>(a, log2N, B, f.log2Ns, tw, log2max, inv);
    else fft_pass_inplace<2>(a, log2N, B, f.log2Ns, tw, log2max, inv);
  }
}

// Moves `total` elements into LDS: ld(e) fetches element e, st(e, v) places
// it.  Each thread issues up to FFT_IO fetches before placing any of them,
// so a block keeps many HBM requests in flight.
template <typename T, typename Ld, typename St>
__device__ __forceinline__ void stage_in(int total, Ld ld, St st) {
  for (int base = 0; base < total; base += NTF * FFT_IO) {
    T v[FFT_IO];
#pragma unroll
    for (int u = 0; u < FFT_IO; ++u) v[u] = ld(min(base + u * NTF + (int)threadIdx.x, total - 1));
#pragma unroll
    for (int u = 0; u < FFT_IO; ++u) {
      const int e = base + u * NTF + (int)threadIdx.x;
      if (e < total) st(e, v[u]);
    }
  }
}

__device__ __forceinline__ void lds_zero(float2* buf, int count) {
  for (int e = threadIdx.x; e < count; e += NTF) buf[e] = make_float2(0.f, 0.f);
}

}  // namespace lam
