// Device helpers shared by the kernel sources: typed loads and stores of
// data / spectra, and the in-place block FFT over LDS.
#pragma once

#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <type_traits>

#include "lamino_common.h"
#include "lamino_internal.h"

namespace lam {

constexpr int NTF = 512;       // threads per block of the FFT kernels
constexpr int LDS_CPLX = 4096; // complex values per FFT block up to 4096 points (32 KB)
constexpr int LDS_CPLX_MAX = 8192;  // the largest transform: one 8192-point block (64 KB)
constexpr int FFT_IO = LDS_CPLX / NTF;  // loads in flight per thread when staging a block

// Complex values an FFT block holds for transforms of N points (the
// kernels' dynamic LDS is this many float2 values, several transforms back
// to back up to 4096 points).
__host__ __device__ __forceinline__ int fft_capacity(int N) { return N > LDS_CPLX ? N : LDS_CPLX; }

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

// The same loads with the element type DT fixed at compile time.  With a
// run-time type each load sits in its own branch and a 16-bit load is
// converted, after a wait for it, inside that branch, so a run of loads
// completes one memory latency at a time; hot loops therefore pick the type
// once (with_storage / with_data) and use these.
template <int DT>
__device__ __forceinline__ float2 ld_ct(const void* p, size_t i) {
  if constexpr (DT == LAMINO_F32) return reinterpret_cast<const float2*>(p)[i];
  else if constexpr (DT == LAMINO_F16) return __half22float2(reinterpret_cast<const __half2*>(p)[i]);
  else return __bfloat1622float2(reinterpret_cast<const __hip_bfloat162*>(p)[i]);
}
template <int DT>
__device__ __forceinline__ void st_ct(void* p, size_t i, float2 v) {
  if constexpr (DT == LAMINO_F32) reinterpret_cast<float2*>(p)[i] = v;
  else if constexpr (DT == LAMINO_F16) reinterpret_cast<__half2*>(p)[i] = __float22half2_rn(v);
  else reinterpret_cast<__hip_bfloat162*>(p)[i] = __float22bfloat162_rn(v);
}
template <int DT>
__device__ __forceinline__ float ld_rt(const void* p, size_t i) {
  if constexpr (DT == LAMINO_F32) return reinterpret_cast<const float*>(p)[i];
  else if constexpr (DT == LAMINO_U8) return (float)reinterpret_cast<const unsigned char*>(p)[i];
  else if constexpr (DT == LAMINO_U16) return (float)reinterpret_cast<const unsigned short*>(p)[i];
  else if constexpr (DT == LAMINO_F16) return __half2float(reinterpret_cast<const __half*>(p)[i]);
  else return __bfloat162float(reinterpret_cast<const __hip_bfloat16*>(p)[i]);
}
// A complex element of storage type DT as loaded (float2, or a 32-bit pair
// of 16-bit values), converted only where it is used, so that a load can
// stay in flight across other work.
template <int DT>
using StoredC = typename std::conditional<DT == LAMINO_F32, float2, unsigned>::type;
template <int DT>
__device__ __forceinline__ StoredC<DT> ld_bits(const void* p, size_t i) {
  return reinterpret_cast<const StoredC<DT>*>(p)[i];
}
template <int DT>
__device__ __forceinline__ float2 bits_c(StoredC<DT> b) {
  if constexpr (DT == LAMINO_F32) return b;
  else if constexpr (DT == LAMINO_F16) return __half22float2(__builtin_bit_cast(__half2, b));
  else return make_float2(__uint_as_float(b << 16), __uint_as_float(b & 0xFFFF0000u));
}
template <int DT>
struct TypeTag {
  static constexpr int value = DT;
};
// f(TypeTag<DT>) for the storage type dt of spectra / slab planes
template <class F>
__device__ __forceinline__ void with_storage(int dt, F&& f) {
  if (dt == LAMINO_F32) f(TypeTag<LAMINO_F32>{});
  else if (dt == LAMINO_F16) f(TypeTag<LAMINO_F16>{});
  else f(TypeTag<LAMINO_BF16>{});
}
// f(TypeTag<DT>) for the element type dt of detector data
template <class F>
__device__ __forceinline__ void with_data(int dt, F&& f) {
  if (dt == LAMINO_F32) f(TypeTag<LAMINO_F32>{});
  else if (dt == LAMINO_U8) f(TypeTag<LAMINO_U8>{});
  else if (dt == LAMINO_U16) f(TypeTag<LAMINO_U16>{});
  else if (dt == LAMINO_F16) f(TypeTag<LAMINO_F16>{});
  else f(TypeTag<LAMINO_BF16>{});
}

// Line integral from raw counts (recording model raw = exp(-d)(flat - dark)
// + dark): -log of the flat/dark-corrected ratio, clamped below at min_ratio;
// a pixel with flat <= dark takes min_ratio.
// (The division runs for every pixel and the result is selected afterwards,
// so that no branch separates a staging loop's loads from their use.)
__device__ __forceinline__ float flat_dark_log(float raw, float dark, float flat, float min_ratio) {
  const float den = flat - dark;
  const float q = (raw - dark) / (den > 0.f ? den : 1.f);
  const float ratio = den > 0.f ? q : min_ratio;
  return -logf(fmaxf(ratio, min_ratio));
}

// ------------------------------------------------------------ block FFT
// Order of this wave's LDS accesses (they execute in issue order) without a
// block barrier: wait for the wave's outstanding LDS operations, and keep the
// compiler from moving memory accesses across.
__device__ __forceinline__ void wave_lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// One Stockham pass of radix R over B transforms of length N = 2^log2N in
// place: each thread reads one butterfly's inputs, twiddles and transforms
// them in registers, and writes the outputs after a barrier (a wave-level
// wait when one wave owns each transform).  N / R <= NTF, so a round covers
// NTF R / N whole transforms.
// The same pass when a transform has more butterflies than the block has
// threads (N = 8192): each thread takes REPS butterflies j = t + NTF rep,
// reads all of them, and writes after the barrier.
template <int R, int REPS>
__device__ __forceinline__ void fft_pass_wide(float2* a, int log2N, int B, int log2Ns,
                                              const float2* __restrict__ tw, int log2max, bool inv) {
  const int N = 1 << log2N;
  const int t = threadIdx.x;
  for (int bb = 0; bb < B; ++bb) {
    float2 v[REPS][R];
#pragma unroll
    for (int rep = 0; rep < REPS; ++rep) {
      const int j = t + rep * NTF;
      if constexpr (R == 8) {
        r8_load(a + bb * N, N, j, v[rep]);
        r8_compute(j, log2Ns, tw, log2max, inv, v[rep]);
      } else if constexpr (R == 4) {
        r4_load(a + bb * N, N, j, v[rep]);
        r4_compute(j, log2Ns, tw, log2max, inv, v[rep]);
      } else {
        r2_load(a + bb * N, N, j, v[rep]);
        r2_compute(j, log2Ns, tw, log2max, inv, v[rep]);
      }
    }
    __syncthreads();
#pragma unroll
    for (int rep = 0; rep < REPS; ++rep) rstore<R>(a + bb * N, t + rep * NTF, log2Ns, v[rep]);
    __syncthreads();
  }
}

template <int R, bool WIDE>
__device__ __forceinline__ void fft_pass_inplace(float2* a, int log2N, int B, int log2Ns,
                                                 const float2* __restrict__ tw, int log2max,
                                                 bool inv, bool wave_local) {
  constexpr int LR = R == 8 ? 3 : (R == 4 ? 2 : 1);
  const int N = 1 << log2N;
  const int lper = log2N - LR;
  const int per = 1 << lper;
  if constexpr (WIDE) {
    if (per > NTF) {  // N = 8192: 1024 (radix 8) or 4096 (radix 2) butterflies
      if constexpr (R == 8) fft_pass_wide<8, LDS_CPLX_MAX / 8 / NTF>(a, log2N, B, log2Ns, tw, log2max, inv);
      else if constexpr (R == 4) fft_pass_wide<4, LDS_CPLX_MAX / 4 / NTF>(a, log2N, B, log2Ns, tw, log2max, inv);
      else fft_pass_wide<2, LDS_CPLX_MAX / 2 / NTF>(a, log2N, B, log2Ns, tw, log2max, inv);
      return;
    }
  }
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
    if (wave_local) wave_lds_sync();
    else __syncthreads();
    if (act) rstore<R>(a + bb * N, j, log2Ns, v);
    if (wave_local) wave_lds_sync();
    else __syncthreads();
  }
}

// B transforms of length 2^log2N stored back to back in LDS at `a`
// (B * N <= fft_capacity(N)), transformed in place.  LOGN > 0 fixes log2N at
// compile time (the passes unroll, their index arithmetic folds); LOGN = 0
// takes log2N at run time (N <= LDS_CPLX).  N > LDS_CPLX (8192 points) has
// its own instantiation: its wide passes hold 16 values per thread, which
// would cost every other transform size its occupancy.
template <int LOGN, int P>
__device__ __forceinline__ void block_fft_fixed(float2* a, int B, const float2* __restrict__ tw,
                                                int log2max, bool inv) {
  if constexpr (P < fft_num_passes(LOGN)) {
    constexpr FftPass f = fft_pass(LOGN, P);
    // N = 8, 64, 512: every pass is radix 8 with at most 64 butterflies per
    // transform, so one wave owns each transform in every pass and the
    // passes need no block barrier
    constexpr bool wave_local = LOGN % 3 == 0 && LOGN <= 9;
    fft_pass_inplace<f.radix, (LOGN > 12)>(a, LOGN, B, f.log2Ns, tw, log2max, inv, wave_local);
    block_fft_fixed<LOGN, P + 1>(a, B, tw, log2max, inv);
  }
}

template <int LOGN>
__device__ inline void block_fft(float2* a, int log2N, int B, const float2* __restrict__ tw, int log2max,
                          bool inv) {
  if constexpr (LOGN > 0) {
    block_fft_fixed<LOGN, 0>(a, B, tw, log2max, inv);
    if constexpr (LOGN % 3 == 0 && LOGN <= 9) __syncthreads();  // the caller reads across transforms
  } else {
    const int np = fft_num_passes(log2N);
    const bool wave_local = log2N % 3 == 0 && log2N <= 9;
    for (int p = 0; p < np; ++p) {
      const FftPass f = fft_pass(log2N, p);
      if (f.radix == 8) fft_pass_inplace<8, false>(a, log2N, B, f.log2Ns, tw, log2max, inv, wave_local);
      else if (f.radix == 4) fft_pass_inplace<4, false>(a, log2N, B, f.log2Ns, tw, log2max, inv, wave_local);
      else fft_pass_inplace<2, false>(a, log2N, B, f.log2Ns, tw, log2max, inv, wave_local);
    }
    if (wave_local) __syncthreads();  // the caller reads across transforms
  }
}

// ------------------------------------------------------ wave-level FFT
// A transform of N = 64 R points (R = 8 or 16) held by one wave, R values
// per lane: lane j holds x[j + 64 r] (r < R).  With n = 64 n1 + n2 and
// k = k1 + R k2, an R-point DFT over n1 = r and the twiddles w^(j k1) give
// Y[k1][j] (w = exp(-+2 pi i / N)); the 64-point DFTs over n2 = 8 m1 + m2
// follow as 8 x 8: an exchange through LDS hands lane (k, m2) =
// (L >> 3, L & 7) the values Y[k1][8 m1 + m2] (m1 = 0..7) of k1 = k + 8 i
// (i < R / 8), whose 8-point DFTs over m1 and twiddles w64^(m2 l1) give
// Z[k1][l1][m2]; a second exchange hands lane (k, l1) = (L >> 3, L & 7) the
// values Z[k1][l1][m2] (m2 = 0..7), and their 8-point DFTs over m2 are
// X[k1 + R l1 + 8 R l2] (l2 = 0..7).  (For R = 16 the second exchange hands
// lane L the pairs (k1, l1) = (L & 15, (L >> 4) + 4 j) instead, so that
// each output register holds 64 consecutive entries.)  The exchange buffers
// hold element (k1, n2) at 72 k1 + n2 and (k1, l1, m2) at 72 k1 + 9 l1 + m2
// (R = 8) or 65 k1 + 16 l1 + 2 m2 (R = 16); searched over linear layouts,
// these spread every write and read of both exchanges over distinct LDS
// banks for R = 8, and leave a few two-way conflicts in the second exchange
// for R = 16 (checked for 16- and 32-lane bank groups of 8-byte values).
__host__ __device__ constexpr int wfft_xch(int R) { return 72 * R; }  // exchange buffer (float2)

template <int R>
struct WaveTw {
  float2 a[R - 1];  // w^(j k1), k1 = 1 .. R-1, j = lane
  float2 b[7];      // w64^(m2 l1), l1 = 1 .. 7, m2 = lane & 7
};

// The lane's twiddles.  With TWL, twa (an LDS table of (R - 1) x 64 values) the
// first-stage twiddles w^(j k1) are kept there instead of in registers, at
// twa[(k1 - 1) 64 + lane]: each lane reads only the entries it wrote, so the
// table needs no barrier, and the waves of a block may share it (they write
// the same values).
template <int R, bool TWL = false>
__device__ __forceinline__ void wave_tw(const float2* __restrict__ tw, int log2max, bool inv,
                                        WaveTw<R>& t, float2* twa = nullptr) {
  constexpr int N = 64 * R;
  constexpr int LOGN = R == 8 ? 9 : 10;
  const int L = threadIdx.x & 63;
#pragma unroll
  for (int k = 1; k < R; ++k) {
    const float2 a = twiddle(tw, ((L * k) & (N - 1)) << (log2max - LOGN), inv);
    if constexpr (TWL) twa[(k - 1) * 64 + L] = a;
    else t.a[k - 1] = a;
  }
#pragma unroll
  for (int k = 1; k < 8; ++k) t.b[k - 1] = twiddle(tw, (((L & 7) * k) & 63) << (log2max - 6), inv);
}

// R-point DFT in registers, natural order in and out (R = 8 or 16: two
// 8-point DFTs of the even and odd inputs combined with w16^k)
template <int R>
__device__ __forceinline__ void dft_reg(float2 v[R], bool inv) {
  if constexpr (R == 8) {
    r8_compute(0, 0, nullptr, 0, inv, v);  // Ns = 1: the plain 8-point DFT
  } else {
    float2 e[8], o[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      e[r] = v[2 * r];
      o[r] = v[2 * r + 1];
    }
    r8_compute(0, 0, nullptr, 0, inv, e);
    r8_compute(0, 0, nullptr, 0, inv, o);
    // w16^k = cos(k pi / 8) -+ i sin(k pi / 8)
    const float c[8] = {1.f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f,
                        0.f, -0.38268343236508977f, -0.70710678118654752f, -0.92387953251128674f};
    const float sk[8] = {0.f, 0.38268343236508977f, 0.70710678118654752f, 0.92387953251128674f,
                         1.f, 0.92387953251128674f, 0.70710678118654752f, 0.38268343236508977f};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float cs = c[k], sn = inv ? sk[k] : -sk[k];
      const float2 t = make_float2(o[k].x * cs - o[k].y * sn, o[k].x * sn + o[k].y * cs);
      v[k] = cadd(e[k], t);
      v[k + 8] = csub(e[k], t);
    }
  }
}

// Output register q of lane L holds X[wave_out<R>(L, q)]: for R = 8 lane
// (k1, l1) = (L >> 3, L & 7) holds X[k1 + 8 l1 + 64 q]; for R = 16 lane
// (k1, l1) = (L & 15, (L >> 4) + 4 j) holds X[k1 + 16 l1 + 128 l2] in
// register 8 j + l2, i.e. X[L + 64 j + 128 l2].
template <int R>
__device__ __forceinline__ int wave_out(int L, int q) {
  if constexpr (R == 8) return (L >> 3) + 8 * (L & 7) + 64 * q;
  return L + 64 * (q >> 3) + 128 * (q & 7);
}

// In place on v: on entry lane j holds x[j + 64 r] in v[r]; on exit lane L
// holds X[wave_out<R>(L, q)] in v[q].  xch: this wave's wfft_xch(R)-value
// buffer; twa: the first-stage twiddle table if wave_tw filled one.
template <int R, bool TWL = false>
__device__ __forceinline__ void wave_fft(float2 v[R], float2* xch, const WaveTw<R>& t, bool inv,
                                         const float2* twa = nullptr) {
  const int L = threadIdx.x & 63;
  const int hi = L >> 3, lo = L & 7;
  dft_reg<R>(v, inv);
#pragma unroll
  for (int k = 1; k < R; ++k) {
    if constexpr (TWL) v[k] = cmul(v[k], twa[(k - 1) * 64 + L]);
    else v[k] = cmul(v[k], t.a[k - 1]);
  }
#pragma unroll
  for (int k = 0; k < R; ++k) xch[72 * k + L] = v[k];
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < R / 8; ++i)
#pragma unroll
    for (int m = 0; m < 8; ++m) v[8 * i + m] = xch[72 * (hi + 8 * i) + 8 * m + lo];
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < R / 8; ++i) {
    r8_compute(0, 0, nullptr, 0, inv, v + 8 * i);
#pragma unroll
    for (int k = 1; k < 8; ++k) v[8 * i + k] = cmul(v[8 * i + k], t.b[k - 1]);
  }
  if constexpr (R == 8) {
#pragma unroll
    for (int k = 0; k < 8; ++k) xch[72 * hi + 9 * k + lo] = v[k];
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = xch[72 * hi + 9 * lo + m];
  } else {
    // R = 16: lane L takes (k1, l1) = (L & 15, (L >> 4) + 4 j), so that each
    // output register covers 64 consecutive entries
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int k = 0; k < 8; ++k) xch[65 * (hi + 8 * i) + 16 * k + 2 * lo] = v[8 * i + k];
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int m = 0; m < 8; ++m) v[8 * j + m] = xch[65 * (L & 15) + 16 * ((L >> 4) + 4 * j) + 2 * m];
  }
  wave_lds_sync();
#pragma unroll
  for (int i = 0; i < R / 8; ++i) r8_compute(0, 0, nullptr, 0, inv, v + 8 * i);
}

// Moves `total` elements into LDS: ld(e) fetches element e, st(e, v) places
// it.  Each thread issues up to IO fetches before placing any of them,
// so a block keeps many HBM requests in flight.  Whole rounds place their
// values with no bounds test: a test per value lets the compiler sink each
// fetch into its own branch, where the fetch is waited for at once.  (ld
// should be branch-free for the same reason: clamp, fetch, then select.)
template <typename T, int IO = FFT_IO, typename Ld, typename St>
__device__ __forceinline__ void stage_in(int total, Ld ld, St st) {
  for (int base = 0; base < total; base += NTF * IO) {
    T v[IO];
#pragma unroll
    for (int u = 0; u < IO; ++u) v[u] = ld(min(base + u * NTF + (int)threadIdx.x, total - 1));
    if (base + NTF * IO <= total) {
#pragma unroll
      for (int u = 0; u < IO; ++u) st(base + u * NTF + (int)threadIdx.x, v[u]);
    } else {
#pragma unroll
      for (int u = 0; u < IO; ++u) {
        const int e = base + u * NTF + (int)threadIdx.x;
        if (e < total) st(e, v[u]);
      }
    }
  }
}

__device__ __forceinline__ void lds_zero(float2* buf, int count) {
  for (int e = threadIdx.x; e < count; e += NTF) buf[e] = make_float2(0.f, 0.f);
}

}  // namespace lam
