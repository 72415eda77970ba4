// gfx950 kernels of the Fourier-route laminography operators.
//
// Backprojection / FBP (eq:fftadj with the filter of eq:recon):
//   proj_cols_fwd  per projection: real column pairs -> h_p-point FFT along v
//   proj_rows_fwd  per (projection, l): w_p-point FFT along u, filter,
//                  store the spectrum slab-major D[l][theta][k]
//   spread         per (slab, 32 x 32 tile): Gaussian gridding of the slab's
//                  samples as rank-16 updates on the matrix cores, no atomics
//   grid_rows_inv  per slab row: inverse N_g-point FFT along x1, crop
//   grid_cols_adj  per slab column block: inverse FFT along x2, crop, psi
//                  correction, store g[l][y][x]
//   x3_adj         vol[z][col] = Re sum_l w_l exp(2 pi i x3 l cos(phi)/h_p) g[l][col]
//                  as a real matrix product on the matrix cores
// Forward projection (eq:fftfwd) runs the transposes in reverse order:
//   x3_fwd, grid_cols_fwd, grid_rows_fwd, interp, proj_rows_inv, proj_cols_inv.
//
// FFTs are in-place Stockham radix-8/4/2 passes over LDS with twiddles from
// a table computed in double precision on the host.  Accumulation is
// float32 throughout; the matrix-core products take 16-bit operands (bf16
// hi + lo splits for float32 data); stored spectra and slab planes may be
// float16 / bfloat16.
#include <cmath>
#include <type_traits>

#include "lamino_common.h"
#include "lamino_device.h"
#include "lamino_internal.h"

namespace lam {

constexpr int NT = 256;        // threads per block (x3 transform, interpolation)
constexpr int TILE_MAX = 64;   // largest interpolation tile edge

constexpr int WFFT_WAVES = 4;  // waves per block of the wave-level row FFT kernels
constexpr int WFFT_ROWS = 4;   // rows per wave
// columns per block of the wave-level column FFT kernels: detector columns
// (real input, measured faster at 8) and slab columns of 512 points
// (measured faster at 16); 1024-point slab columns take 8 (16 would need
// 148 KB of LDS per block)
constexpr int WFFT_CW_DET = 8;
constexpr int WFFT_CW_SLAB = 16;
constexpr int WFFT_CW_WIDE = 8;

// ====================================================== detector transforms
// W1 layout: [theta_local][n_slab][w] float2.

// Column pairs (c, c+1) of projection theta0 + blockIdx.y packed as one
// complex h_p-point FFT along v; the two real spectra are separated by
// Hermitian symmetry and the half l = 0 .. n_slab-1 is stored.
// data holds projections data_th0 .. (a whole input or a streamed chunk).
// f(TypeTag<data type>, TypeTag<raw counts>) for the detector data of a
// call: raw counts take the dark / flat correction and -log on loading
template <class F>
__device__ __forceinline__ void with_data_raw(const KParams& p, F&& f) {
  with_data(p.data_dtype, [&](auto ty) {
    if (p.dark) f(ty, TypeTag<1>{});
    else f(ty, TypeTag<0>{});
  });
}

template <int LOGN>
__global__ __launch_bounds__(NTF) void k_proj_cols_fwd(KParams p, const void* __restrict__ data,
                                                      float2* __restrict__ w1, int theta0,
                                                      int cp, int data_th0) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int tl = blockIdx.y;
  const int th = theta0 + tl;
  const int c0 = blockIdx.x * 2 * cp;
  const int hp = p.h_p;
  lds_zero(buf, cp * hp);
  __syncthreads();
  const int wide = 2 * cp;
  const float iwide = 1.f / (float)wide;
  float* bf = reinterpret_cast<float*>(buf);
  const size_t row0 = (size_t)(th - data_th0) * p.h;
  const float fin = p.dyn ? p.dyn[0] : 1.f;  // float16 storage: input factor of the call
  with_data_raw(p, [&](auto ty, auto raw) {
    stage_in<float>(
        p.h * wide,
        [&](int e) {
          const int r = div24(e, wide, iwide), c = c0 + e - r * wide;
          const int cs = min(c, p.w - 1);  // past the detector: a valid load, dropped below
          float v = ld_rt<decltype(ty)::value>(data, (row0 + r) * p.w + cs);
          if constexpr (decltype(raw)::value) {
            const size_t q = (size_t)r * p.w + cs;
            v = flat_dark_log(v, p.dark[q], p.flat[q], p.min_ratio);
          }
          // (a factor, not a select: a select of a loaded value lets the compiler move
          // the load into a branch, where it is waited for at once)
          return v * (c < p.w ? fin : 0.f);
        },
        [&](int e, float v) {
          const int r = div24(e, wide, iwide), cl = e - r * wide;
          bf[2 * ((cl >> 1) * hp + ((r - p.h / 2) & (hp - 1))) + (cl & 1)] = v;
        });
  });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_hp, cp, p.tw, p.log2_twmax, false);
  const float2* res = buf;
  const size_t base = (size_t)tl * p.n_slab * p.w;
  for (int e = threadIdx.x; e < p.n_slab * wide; e += NTF) {
    const int l = div24(e, wide, iwide), cl = e - l * wide;
    const int c = c0 + cl;
    if (c >= p.w) continue;
    const float2* z = res + (cl >> 1) * hp;
    const float2 zl = z[l], zm = cconj(z[(hp - l) & (hp - 1)]);
    float2 x;
    if ((cl & 1) == 0) x = cscale(cadd(zl, zm), 0.5f);        // (Z[l] + conj Z[-l]) / 2
    else x = cscale(mul_mi(csub(zl, zm)), 0.5f);              // (Z[l] - conj Z[-l]) / 2i
    w1[base + (size_t)l * p.w + c] = x;
  }
}

// k_proj_cols_fwd for h_p = N = 64 R (512 or 1024) with one wave per complex column: a block
// stages CW column pairs of one projection (2 CW input columns, contiguous
// rows) into LDS, column-major with stride wcol_stride(R, CW) so that the staging
// stores and every access of the transform fall in distinct banks; each wave
// transforms CW / 8 columns in place (the column's own LDS span is its
// exchange buffer), writes the spectrum back in natural order, and the
// block then separates the two real spectra of each pair and writes rows
// l = 0 .. n_slab-1 of W1, 2 CW consecutive columns per row.
// Column block and projection of a detector column block.  Neighbouring
// column blocks read or write the two 64-byte halves of the same 128-byte
// lines (16 float32 columns each), so each run of 16 dispatched blocks is
// reordered to place column blocks 2k and 2k + 1 at dispatch positions k
// and k + 8: hardware workgroup b runs on XCD b mod 8, and both halves of a
// line then meet in the same XCD's L2.
__device__ __forceinline__ void det_col_block(int& cb, int& tl) {
  const int nb = (int)gridDim.x;
  const int total = nb * (int)gridDim.y;
  int b = (int)(blockIdx.x + gridDim.x * blockIdx.y);
  if ((b | 15) < total) b = (b & ~15) + 2 * (b & 7) + ((b >> 3) & 1);
  cb = b % nb;
  tl = b / nb;
}

constexpr __host__ __device__ int wcol_stride(int R, int cw) { return wfft_xch(R) + 32 / cw; }

template <int R, int CW>
__global__ __launch_bounds__(512) void k_proj_cols_fwd_w(KParams p, const void* __restrict__ data,
                                                         float2* __restrict__ w1, int theta0,
                                                         int data_th0) {
  constexpr int N = 64 * R;
  constexpr int S = wcol_stride(R, CW);
  __shared__ float2 buf[CW * S];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  int cb, tl;
  det_col_block(cb, tl);
  const int th = theta0 + tl;
  const int c0 = cb * 2 * CW;
  float* bf = reinterpret_cast<float*>(buf);
  const size_t row0 = (size_t)(th - data_th0) * p.h;
  const float fin = p.dyn ? p.dyn[0] : 1.f;  // float16 storage: input factor of the call
  with_data_raw(p, [&](auto ty, auto raw) {
    stage_in<float>(
        p.h * 2 * CW,
        [&](int e) {
          const int r = e / (2 * CW), c = c0 + e % (2 * CW);
          const int cs = min(c, p.w - 1);  // past the detector: a valid load, dropped below
          float v = ld_rt<decltype(ty)::value>(data, (row0 + r) * p.w + cs);
          if constexpr (decltype(raw)::value) {
            const size_t q = (size_t)r * p.w + cs;
            v = flat_dark_log(v, p.dark[q], p.flat[q], p.min_ratio);
          }
          // (a factor, not a select: a select of a loaded value lets the compiler move
          // the load into a branch, where it is waited for at once)
          return v * (c < p.w ? fin : 0.f);
        },
        [&](int e, float v) {
          const int r = e / (2 * CW), cl = e % (2 * CW);
          bf[2 * ((cl >> 1) * S + ((r - p.h / 2) & (N - 1))) + (cl & 1)] = v;
        });
  });
  WaveTw<R> t;
  wave_tw<R>(p.tw, p.log2_twmax, false, t);
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < CW / 8; ++cc) {
    float2* col = buf + (wv * (CW / 8) + cc) * S;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = L + 64 * r;  // entry (row - h/2) mod N holds detector row `row`
      v[r] = ((pos + p.h / 2) & (N - 1)) < p.h ? col[pos] : make_float2(0.f, 0.f);
    }
    wave_fft<R>(v, col, t, false);
#pragma unroll
    for (int q = 0; q < R; ++q) col[wave_out<R>(L, q)] = v[q];
  }
  __syncthreads();
  const size_t base = (size_t)tl * p.n_slab * p.w;
  for (int e = threadIdx.x; e < p.n_slab * 2 * CW; e += 512) {
    const int l = e / (2 * CW), cl = e % (2 * CW);
    const int c = c0 + cl;
    if (c >= p.w) continue;
    const float2* z = buf + (cl >> 1) * S;
    const float2 zl = z[l], zm = cconj(z[(N - l) & (N - 1)]);
    float2 x;
    if ((cl & 1) == 0) x = cscale(cadd(zl, zm), 0.5f);        // (Z[l] + conj Z[-l]) / 2
    else x = cscale(mul_mi(csub(zl, zm)), 0.5f);              // (Z[l] - conj Z[-l]) / 2i
    w1[base + (size_t)l * p.w + c] = x;
  }
}

// Rows l of the column spectra: w_p-point FFT along u, times the transfer
// function, stored as D[l][theta - d_th0][k] (k = m mod w_p) with d_nth
// projections per slab (all of them, or one streamed chunk).
template <int LOGN>
__global__ __launch_bounds__(NTF) void k_proj_rows_fwd(KParams p, const float2* __restrict__ w1,
                                                      void* __restrict__ D, const float* __restrict__ filt,
                                                      const float2* __restrict__ phase, int theta0,
                                                      int rows, int d_nth, int d_th0) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int tl = blockIdx.y;
  const int th = theta0 + tl;
  const int l0 = blockIdx.x * rows;
  const int wp = p.w_p;
  lds_zero(buf, rows * wp);
  __syncthreads();
  const size_t base = (size_t)tl * p.n_slab * p.w;
  const int nr = min(rows, p.n_slab - l0);
  const float iw = 1.f / (float)p.w;
  stage_in<float2>(
      nr * p.w, [&](int e) { return w1[base + (size_t)l0 * p.w + e]; },
      [&](int e, float2 v) {
        const int b = div24(e, p.w, iw), c = e - b * p.w;
        buf[b * wp + ((c - p.w / 2) & (wp - 1))] = v;
      });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_wp, rows, p.tw, p.log2_twmax, false);
  const float2* res = buf;
  // four elements per thread at a time: their transfer-function (and phase)
  // loads are issued together, the stores follow
  const int total = rows * wp;
  with_storage(p.storage_dtype, [&](auto ty) {
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * NTF) {
      float2 v[4];
      if (phase) {  // (a branch per element would wait for each load)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * NTF, total - 1);
          const int k = e & (wp - 1);
          v[u] = cmul(cscale(res[e], filt[k]), phase[k]);
        }
      } else {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = min(e0 + u * NTF, total - 1);
          v[u] = cscale(res[e], filt[e & (wp - 1)]);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * NTF;
        const int l = l0 + (e >> p.log2_wp), k = e & (wp - 1);
        if (e < total && l < p.n_slab)
          st_ct<decltype(ty)::value>(D, ((size_t)l * d_nth + (th - d_th0)) * wp + k, v[u]);
      }
    }
  });
}


// k_proj_rows_fwd for w_p = N = 64 R (512 or 1024) with one wave per row: the padded row is
// loaded straight into the lanes (lane j: entries j + 64 r), transformed by
// wave_fft and written to D with the transfer function; each wave takes
// rows_per_wave consecutive rows.
template <int R>
__global__ __launch_bounds__(64 * WFFT_WAVES) void k_proj_rows_fwd_w(
    KParams p, const float2* __restrict__ w1, void* __restrict__ D, const float* __restrict__ filt,
    const float2* __restrict__ phase, int theta0, int rows_per_wave, int d_nth, int d_th0) {
  constexpr int N = 64 * R;
  __shared__ float2 xch_all[WFFT_WAVES * wfft_xch(R)];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  float2* xch = xch_all + wv * wfft_xch(R);
  // 1024-point rows keep the first-stage twiddles in LDS (fewer registers, more waves)
  __shared__ float2 twa_s[R == 16 ? 15 * 64 : 1];
  float2* const twa = R == 16 ? twa_s : nullptr;
  // projections in reverse order: the column pass wrote the last ones last,
  // and the Infinity Cache still holds them
  const int tl = (int)gridDim.y - 1 - (int)blockIdx.y;
  const int th = theta0 + tl;
  WaveTw<R> t;
  wave_tw<R, R == 16>(p.tw, p.log2_twmax, false, t, twa);
  // the transfer function at this lane's outputs: registers, or (R = 16)
  // this lane's own entries of an LDS table
  __shared__ float f_s[R == 16 ? 16 * 64 : 1];
  float f[R == 16 ? 1 : R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    if constexpr (R == 16) f_s[q * 64 + L] = filt[wave_out<R>(L, q)];
    else f[q] = filt[wave_out<R>(L, q)];
  }
  const float2* src = w1 + (size_t)tl * p.n_slab * p.w;
  const int l0 = (blockIdx.x * WFFT_WAVES + wv) * rows_per_wave;
  const int l1 = min(l0 + rows_per_wave, p.n_slab);
  with_storage(p.storage_dtype, [&](auto ty) {
    for (int l = l0; l < l1; ++l) {
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int c = (L + 64 * r + p.w / 2) & (N - 1);  // entry (c - w/2) mod w_p holds column c
        v[r] = c < p.w ? src[(size_t)l * p.w + c] : make_float2(0.f, 0.f);
      }
      wave_fft<R, R == 16>(v, xch, t, false, twa);
      const size_t o = ((size_t)l * d_nth + (th - d_th0)) * N;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        float2 x = cscale(v[q], R == 16 ? f_s[q * 64 + L] : f[q]);
        if (phase) x = cmul(x, phase[wave_out<R>(L, q)]);
        st_ct<decltype(ty)::value>(D, o + wave_out<R>(L, q), x);
      }
    }
  });
}

// Rotation-axis offset: exp(2 pi i m delta / w_p) for k = m mod w_p, in
// double precision (a translation of the rows by delta columns).
__global__ void k_axis_phase(float2* __restrict__ out, int wp, double delta) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= wp) return;
  const int m = k < wp / 2 ? k : k - wp;
  double sn, cs;
  sincospi(2.0 * m * delta / wp, &sn, &cs);
  out[k] = make_float2((float)cs, (float)sn);
}

// Inverse of the row step (forward projection): D[l][theta][.] -> inverse
// FFT along m -> detector columns, W1[theta_local][l][c].
template <int LOGN>
__global__ __launch_bounds__(NTF) void k_proj_rows_inv(KParams p, const void* __restrict__ D,
                                                      float2* __restrict__ w1, int theta0,
                                                      int rows) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int tl = blockIdx.y;
  const int th = theta0 + tl;
  const int l0 = blockIdx.x * rows;
  const int wp = p.w_p;
  with_storage(p.storage_dtype, [&](auto ty) {
    stage_in<float2>(
        rows * wp,
        [&](int e) {
          const int b = e >> p.log2_wp, k = e & (wp - 1);
          const int l = l0 + b;
          // rows past the last slab drop out; the Nyquist bin is not part of the
          // sum (and may never have been written: its neighbour is read instead);
          // a factor rather than a select, which would move the load into a branch
          const int kr = k == (wp >> 1) ? k - 1 : k;
          const float2 v = ld_ct<decltype(ty)::value>(D, ((size_t)min(l, p.n_slab - 1) * p.n_theta + th) * wp + kr);
          return cscale(v, l < p.n_slab && k != (wp >> 1) ? 1.f : 0.f);
        },
        [&](int e, float2 v) { buf[e] = v; });
  });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_wp, rows, p.tw, p.log2_twmax, true);
  const float2* res = buf;
  const size_t base = (size_t)tl * p.n_slab * p.w;
  const float iw = 1.f / (float)p.w;
  for (int e = threadIdx.x; e < rows * p.w; e += NTF) {
    const int b = div24(e, p.w, iw), c = e - b * p.w;
    const int l = l0 + b;
    if (l < p.n_slab) w1[base + (size_t)l * p.w + c] = res[b * wp + ((c - p.w / 2) & (wp - 1))];
  }
}

// Inverse of the column step: the half spectra of columns (c, c+1) are
// completed by Hermitian symmetry (Nyquist bin zero, imaginary part of
// l = 0 dropped), packed as Z = X_c + i X_{c+1}, inverse transformed along
// v, and the real / imaginary parts scaled by 1/(h_p w_p) give the two
// detector columns.
template <int LOGN>
__global__ __launch_bounds__(NTF) void k_proj_cols_inv(KParams p, const float2* __restrict__ w1,
                                                      void* __restrict__ data, int theta0,
                                                      int cp, float scale) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int tl = blockIdx.y;
  const int th = theta0 + tl;
  const int c0 = blockIdx.x * 2 * cp;
  const int hp = p.h_p;
  lds_zero(buf, cp * hp);
  __syncthreads();
  const size_t base = (size_t)tl * p.n_slab * p.w;
  const float icp = 1.f / (float)cp;
  stage_in<float4>(
      p.n_slab * cp,
      [&](int e) {
        const int l = div24(e, cp, icp), pp = e - l * cp;
        const int ca = c0 + 2 * pp, cb = ca + 1;
        const float2 xa = ca < p.w ? w1[base + (size_t)l * p.w + ca] : make_float2(0.f, 0.f);
        const float2 xb = cb < p.w ? w1[base + (size_t)l * p.w + cb] : make_float2(0.f, 0.f);
        return make_float4(xa.x, xa.y, xb.x, xb.y);
      },
      [&](int e, float4 x) {
        const int l = div24(e, cp, icp), pp = e - l * cp;
        float2* z = buf + pp * hp;
        // x = (Re X_a, Im X_a, Re X_b, Im X_b)
        if (l == 0) {
          z[0] = make_float2(x.x, x.z);
        } else {
          z[l] = make_float2(x.x - x.w, x.y + x.z);
          z[hp - l] = make_float2(x.x + x.w, x.z - x.y);
        }
      });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_hp, cp, p.tw, p.log2_twmax, true);
  const float2* res = buf;
  const int wide = 2 * cp;
  const float iwide = 1.f / (float)wide;
  const float* bf = reinterpret_cast<const float*>(res);
  const float out = scale * (p.dyn ? p.dyn[1] : 1.f);
  for (int e = threadIdx.x; e < p.h * wide; e += NTF) {
    const int r = div24(e, wide, iwide), cl = e - r * wide;
    const int c = c0 + cl;
    if (c >= p.w) continue;
    const int pos = (r - p.h / 2) & (hp - 1);
    st_r(data, ((size_t)th * p.h + r) * p.w + c, bf[2 * ((cl >> 1) * hp + pos) + (cl & 1)] * out,
         p.data_dtype);
  }
}

// k_proj_rows_inv for w_p = N = 64 R (512 or 1024) with one wave per row (wave_fft).
template <int R>
__global__ __launch_bounds__(64 * WFFT_WAVES) void k_proj_rows_inv_w(KParams p, const void* __restrict__ D,
                                                                     float2* __restrict__ w1, int theta0,
                                                                     int rows_per_wave) {
  constexpr int N = 64 * R;
  __shared__ float2 xch_all[WFFT_WAVES * wfft_xch(R)];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  float2* xch = xch_all + wv * wfft_xch(R);
  // 1024-point rows keep the first-stage twiddles in LDS (fewer registers, more waves)
  __shared__ float2 twa_s[R == 16 ? 15 * 64 : 1];
  float2* const twa = R == 16 ? twa_s : nullptr;
  const int tl = blockIdx.y;
  const int th = theta0 + tl;
  WaveTw<R> t;
  wave_tw<R, R == 16>(p.tw, p.log2_twmax, true, t, twa);
  float2* dst = w1 + (size_t)tl * p.n_slab * p.w;
  const int l0 = (blockIdx.x * WFFT_WAVES + wv) * rows_per_wave;
  const int l1 = min(l0 + rows_per_wave, p.n_slab);
  with_storage(p.storage_dtype, [&](auto ty) {
    for (int l = l0; l < l1; ++l) {
      const size_t o = ((size_t)l * p.n_theta + th) * N;
      float2 v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // the Nyquist bin (k = N/2, lane 0 of r = R/2) is not part of the sum
        // and may never have been written: that lane reads its neighbour and
        // drops it
        const int k = r == R / 2 && L == 0 ? N / 2 - 1 : L + 64 * r;
        const float2 x = ld_ct<decltype(ty)::value>(D, o + k);
        v[r] = r == R / 2 && L == 0 ? make_float2(0.f, 0.f) : x;
      }
      wave_fft<R, R == 16>(v, xch, t, true, twa);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const int c = (wave_out<R>(L, q) + p.w / 2) & (N - 1);  // entry (c - w/2) mod w_p -> column c
        if (c < p.w) dst[(size_t)l * p.w + c] = v[q];
      }
    }
  });
}

// k_proj_cols_inv for h_p = N = 64 R (512 or 1024) with one wave per complex column: the half
// spectra of CW column pairs are completed by Hermitian symmetry into LDS
// columns (stride wcol_stride(R, CW); the Nyquist entry is zeroed on loading),
// transformed in place by one wave each, and written as 2 CW detector
// columns per row.
template <int R, int CW>
__global__ __launch_bounds__(512) void k_proj_cols_inv_w(KParams p, const float2* __restrict__ w1,
                                                         void* __restrict__ data, int theta0, float scale) {
  constexpr int N = 64 * R;
  constexpr int S = wcol_stride(R, CW);
  __shared__ float2 buf[CW * S];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  int cb, tl;
  det_col_block(cb, tl);
  const int th = theta0 + tl;
  const int c0 = cb * 2 * CW;
  const size_t base = (size_t)tl * p.n_slab * p.w;
  stage_in<float4>(
      p.n_slab * CW,
      [&](int e) {
        const int l = e / CW, pp = e % CW;
        const int ca = c0 + 2 * pp, cb = ca + 1;
        const float2 xa = ca < p.w ? w1[base + (size_t)l * p.w + ca] : make_float2(0.f, 0.f);
        const float2 xb = cb < p.w ? w1[base + (size_t)l * p.w + cb] : make_float2(0.f, 0.f);
        return make_float4(xa.x, xa.y, xb.x, xb.y);
      },
      [&](int e, float4 x) {
        const int l = e / CW, pp = e % CW;
        float2* z = buf + pp * S;
        // x = (Re X_a, Im X_a, Re X_b, Im X_b)
        if (l == 0) {
          z[0] = make_float2(x.x, x.z);
        } else {
          z[l] = make_float2(x.x - x.w, x.y + x.z);
          z[N - l] = make_float2(x.x + x.w, x.z - x.y);
        }
      });
  WaveTw<R> t;
  wave_tw<R>(p.tw, p.log2_twmax, true, t);
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < CW / 8; ++cc) {
    float2* col = buf + (wv * (CW / 8) + cc) * S;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = (r == R / 2 && L == 0) ? make_float2(0.f, 0.f) : col[L + 64 * r];
    wave_fft<R>(v, col, t, true);
#pragma unroll
    for (int q = 0; q < R; ++q) col[wave_out<R>(L, q)] = v[q];
  }
  __syncthreads();
  const float* bf = reinterpret_cast<const float*>(buf);
  const float out = scale * (p.dyn ? p.dyn[1] : 1.f);
  for (int e = threadIdx.x; e < p.h * 2 * CW; e += 512) {
    const int r = e / (2 * CW), cl = e % (2 * CW);
    const int c = c0 + cl;
    if (c >= p.w) continue;
    const int pos = (r - p.h / 2) & (N - 1);
    st_r(data, ((size_t)th * p.h + r) * p.w + c, bf[2 * ((cl >> 1) * S + pos) + (cl & 1)] * out,
         p.data_dtype);
  }
}

// ================================================================ gridding
// Gaussian weights exp(-beta d^2) at the 2M taps d = (1 - M) - f, ..., M - f
// by the recurrence w_{i+1} = w_i r_i, r_{i+1} = r_i exp(-2 beta).
template <int M>
__device__ __forceinline__ void gauss_taps(float f, float beta, float e2b, float w[2 * M]) {
  const float d0 = (float)(1 - M) - f;
  w[0] = __expf(-beta * d0 * d0);
  float r = __expf(-beta * (2.f * d0 + 1.f));
#pragma unroll
  for (int i = 1; i < 2 * M; ++i) {
    w[i] = w[i - 1] * r;
    r *= e2b;
  }
}

// Adjoint USFFT step (3) on the matrix cores.  For one 32 x 32 tile of the
// slab grid, spreading is a sum of rank-one updates
//     G_tile += wy_s (c_s wx_s)^T,
// wy_s / wx_s the sample's Gaussian weights on the tile rows / columns (zero
// outside its 2M taps), so a batch of K samples is one 32 x 32 x K matrix
// product with the tile held in MFMA accumulators.  One wave per tile; the
// launch grid is (slab, tile rank) with slabs varying fastest and tiles in
// centre-out rings, so the densest tiles of every slab start first and the
// sparse outer tiles fill the tail.
//
// Candidates: for each periodic copy of the tile that the slab's samples can
// reach and each pass of 64 angles, lane j finds the m-interval of angle j
// whose Gaussian footprint meets the copy (an exact line / box intersection);
// the non-empty intervals are compacted with a ballot and held one per lane
// (start, first m, angle), and a batch of 64 consecutive candidates locates
// its intervals by a uniform scan over the few interval starts it spans.
//
// Staging: each candidate stores its 2M row weights and 2M column values
// (c times the column weights) in an LDS slot framed by a zero entry on each
// side.  Lane r of the matrix operand needs the tap r - ly of a sample whose
// taps start at tile row ly; the byte offset of that tap is clamped onto the
// slot's zeros, so rows outside the footprint read 0 with no branch.
//
// Precision: float32 storage uses bf16 hi / lo splits (three products per
// component, ~2^-17 relative error); float16 / bfloat16 storage uses one
// float16 / bfloat16 product.
typedef unsigned short v8u __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int SP_T = 32;       // tile edge = MFMA block
constexpr int SP_K = 16;       // samples per matrix product
constexpr int SP_NK = 64;        // staging slots: one batch of candidates

typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));

// bf16(a) | bf16(b) << 16, round to nearest even: one packed conversion
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){a, b}, v2bf));
}
__device__ __forceinline__ unsigned bf16_bits(float x) {
  return (unsigned)__builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ unsigned f16_bits(float x) {
  return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)x);
}
// f16(a w) | f16(b w) << 16, each product rounded once: mixed-precision
// FMAs (float32 sources, zero addend) into the low and the high half
__device__ __forceinline__ unsigned f16_prod_pair(float a, float b, float w) {
  unsigned r;
  asm("v_fma_mixlo_f16 %0, %1, %2, 0\n\tv_fma_mixhi_f16 %0, %3, %2, 0"
      : "=&v"(r)
      : "v"(a), "v"(w), "v"(b));
  return r;
}
// hi | lo << 16 with hi + lo ~ x to ~2^-17 (round-to-nearest conversions);
// hi is converted twice so that the final pair is one conversion of (x, lo)
__device__ __forceinline__ unsigned bf16_split(float x) {
  const float h = __uint_as_float(bf16_pair(x, x) << 16);
  return bf16_pair(x, x - h);
}
// the splits of a complex value: (re hi | re lo << 16, im hi | im lo << 16)
__device__ __forceinline__ uint2 bf16_split2(float re, float im) {
  const unsigned hh = bf16_pair(re, im);
  const float hre = __uint_as_float(hh << 16), him = __uint_as_float(hh & 0xFFFF0000u);
  return make_uint2(bf16_pair(re, re - hre), bf16_pair(im, im - him));
}
__device__ __forceinline__ int med3i(int a, int lo, int hi) {
  int r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(lo), "v"(hi));
  return r;
}

template <int PREC>
__device__ __forceinline__ v16f mfma16(v8u a, v8u b, v16f c) {
  if (PREC == 1)
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, a),
                                                  __builtin_bit_cast(v8h, b), c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, a),
                                                 __builtin_bit_cast(v8bf, b), c, 0, 0, 0);
}

// One candidate sample of a lane: position, local tap-0 cell, value.
// (The value is kept as loaded and converted at staging, so that its load
// stays in flight during the matrix products of the previous batch.)
template <int DT>
struct SpreadCand {
  bool use;
  int lx, ly;
  float X, Y;
  StoredC<DT> c;
};

// PREC 0: bf16 x3 (float32 storage), 1: float16 x1, 2: bfloat16 x1; PREC is
// also the storage type of D
static_assert(LAMINO_F32 == 0 && LAMINO_F16 == 1 && LAMINO_BF16 == 2, "PREC doubles as the storage type");
template <int M, int PREC>
__global__ __launch_bounds__(64) void k_spread(KParams p, const void* __restrict__ D,
                                               float2* __restrict__ G, int slab0, int d_l0, int ns) {
  constexpr int W = 2 * M;
  constexpr int WS = W + 3;  // slot: zero, W taps, zero, pad (an odd stride in 32-bit words)
  // row weight: bf16 hi | lo (PREC 0) or one 16-bit value; column value:
  // (re, im) as hi | lo words (PREC 0) or re | im << 16
  typedef typename std::conditional<PREC == 0, unsigned, unsigned short>::type TA;
  typedef typename std::conditional<PREC == 0, uint2, unsigned>::type TB;
  constexpr int SA = sizeof(TA), SB = sizeof(TB);
  __shared__ __align__(16) int st_l[SP_NK];  // ly * SA (low 16 bits) | lx * SB << 16
  __shared__ TA st_a[64 * WS];
  __shared__ TB st_b[64 * WS];
  const int lane = threadIdx.x;
  const int ntx = p.grid / SP_T;
  // The slabs in two halves, each with its slabs varying fastest and its
  // dense central tiles first: the second half's grids, written last, are
  // still in the Infinity Cache when the row pass, which takes the slabs in
  // reverse order, reads them.
  const int nh = ns >> 1;
  const unsigned first = (unsigned)nh * (unsigned)(ntx * ntx);
  int sl, rank;
  if (blockIdx.x < first) {
    sl = (int)(blockIdx.x % (unsigned)nh);
    rank = (int)(blockIdx.x / (unsigned)nh);
  } else {
    const unsigned b2 = blockIdx.x - first;
    sl = nh + (int)(b2 % (unsigned)(ns - nh));
    rank = (int)(b2 / (unsigned)(ns - nh));
  }
  const int l = slab0 + sl;
  int tx, ty;
  ring_tile(rank, ntx, tx, ty);
  const int X0 = -(p.grid >> 1) + tx * SP_T;
  const int Y0 = -(p.grid >> 1) + ty * SP_T;
  const float gcl = p.gs * (float)l;
  const float e2b = __expf(-2.f * p.beta);
  const int half_m = (p.w_p >> 1) - 1;
  const int r = lane & 31;           // tile row of A / tile column of B held by this lane
  const int kq = (lane >> 5) * 8;    // first of the lane's 8 samples within a group of 16
  // periodic copies of the tile that the slab's samples can reach:
  // |xi_perp| <= sqrt(1/4 + (l sin(phi) / h_p)^2) (eq:uneqspace)
  const float reach = sqrtf(0.25f * (float)p.grid * (float)p.grid + gcl * gcl) + 2.f;
  bool rx[3], ry[3];
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3) {
    const float x0 = (float)(X0 + (s3 - 1) * p.grid - M), y0 = (float)(Y0 + (s3 - 1) * p.grid - M);
    rx[s3] = x0 < reach && x0 + (float)(SP_T + 2 * M) > -reach;
    ry[s3] = y0 < reach && y0 + (float)(SP_T + 2 * M) > -reach;
  }
  for (int k = lane; k < 64; k += 64) {
    st_a[k * WS] = TA{};
    st_a[k * WS + W + 1] = TA{};
    st_b[k * WS] = TB{};
    st_b[k * WS + W + 1] = TB{};
  }
  v16f cre = {}, cim = {};

  for (int sy = -1; sy <= 1; ++sy) {
    if (!ry[sy + 1]) continue;
    for (int sx = -1; sx <= 1; ++sx) {
      if (!rx[sx + 1]) continue;
      const float bx0 = (float)(X0 + sx * p.grid - M), by0 = (float)(Y0 + sy * p.grid - M);
      const int ox = sx * p.grid + X0, oy = sy * p.grid + Y0;  // copy origin
      for (int th0 = 0; th0 < p.n_theta; th0 += 64) {
        const int th = th0 + lane;
        int mlo = 0, mhi = -1;
        const bool found = th < p.n_theta &&
                           tile_candidates(p.ncw, gcl, p.trig[th], bx0, by0, (float)(SP_T + 2 * M - 1),
                                           (float)(SP_T + 2 * M - 1), half_m, mlo, mhi);
        const unsigned long long fm = __ballot(found);
        const int nseg = __popcll(fm);
        if (nseg == 0) continue;
        // compact: found lanes to 0 .. nseg-1 in lane order, the rest after;
        // lane j then holds interval j: length, first m, angle
        const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
        const int dst = 4 * (found ? below : nseg + lane - below);
        const int len = __builtin_amdgcn_ds_permute(dst, found ? mhi - mlo + 1 : 0);
        const int smlo = __builtin_amdgcn_ds_permute(dst, mlo);
        const int sth = __builtin_amdgcn_ds_permute(dst, th);
        const float2 cst = p.trig[min(sth, p.n_theta - 1)];  // interval's angle
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int t = __shfl_up(incl, o);
          if (lane >= o) incl += t;
        }
        const int spre = incl - len;
        const int total = __shfl(incl, 63);
        int jcur = 0;  // interval holding candidate `base`
        // candidate base + lane: interval, position, value
        auto fetch = [&](int base, SpreadCand<PREC>& cd) {
          const int i = base + lane;
          int j = jcur;
          for (int jj = jcur + 1; jj < nseg; ++jj) {
            const int s0 = __builtin_amdgcn_readlane(spre, jj);
            if (s0 > base + 63) break;
            if (s0 <= i) j = jj;
          }
          jcur = __builtin_amdgcn_readlane(j, 63);
          cd.use = false;
          cd.lx = cd.ly = 0;
          cd.X = cd.Y = 0.f;
          cd.c = StoredC<PREC>{};
          const int pj = __shfl(spre, j), mj = __shfl(smlo, j), tj = __shfl(sth, j);
          const float2 cs = make_float2(__shfl(cst.x, j), __shfl(cst.y, j));
          if (i >= total) return;
          const int m = mj + (i - pj);
          sample_pos(p.ncw, gcl, cs, m, cd.X, cd.Y);
          cd.lx = (int)floorf(cd.X) - M + 1 - ox;
          cd.ly = (int)floorf(cd.Y) - M + 1 - oy;
          cd.use = cd.lx + W > 0 && cd.lx < SP_T && cd.ly + W > 0 && cd.ly < SP_T;
          if (cd.use)
            cd.c = ld_bits<PREC>(D, ((size_t)(l - d_l0) * p.n_theta + tj) * p.w_p + (m & (p.w_p - 1)));
        };
        SpreadCand<PREC> cur;
        fetch(0, cur);
        for (int base = 0; base < total; base += 64) {
          // stage the candidates whose taps reach the tile
          const unsigned long long mask = __ballot(cur.use);
          const int cnt = __popcll(mask);
          const int pos = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
          if (cur.use) {
            float wx[W], wy[W];
            const float2 cc = bits_c<PREC>(cur.c);
            gauss_taps<M>(cur.X - floorf(cur.X), p.beta, e2b, wx);
            gauss_taps<M>(cur.Y - floorf(cur.Y), p.beta, e2b, wy);
#pragma unroll
            for (int k = 0; k < W; ++k) {
              if constexpr (PREC == 0) {
                st_a[pos * WS + 1 + k] = bf16_split(wy[k]);
                st_b[pos * WS + 1 + k] = bf16_split2(cc.x * wx[k], cc.y * wx[k]);
              } else if constexpr (PREC == 1) {
                st_a[pos * WS + 1 + k] = (unsigned short)f16_bits(wy[k]);
                st_b[pos * WS + 1 + k] = f16_prod_pair(cc.x, cc.y, wx[k]);
              } else {
                st_a[pos * WS + 1 + k] = (unsigned short)bf16_bits(wy[k]);
                st_b[pos * WS + 1 + k] = bf16_pair(cc.x * wx[k], cc.y * wx[k]);
              }
            }
            st_l[pos] = (int)(((unsigned)(cur.ly * SA) & 0xFFFFu) | ((unsigned)(cur.lx * SB) << 16));
          }
          // padding samples of the last group read only zeros
          if (lane < SP_K && cnt + lane < 64)
            st_l[cnt + lane] = (int)(((unsigned)(-1024 * SA) & 0xFFFFu) | ((unsigned)(-1024 * SB) << 16));
          __syncthreads();
          // the next batch's loads are in flight during the products below
          fetch(base + 64, cur);
          for (int g0 = 0; g0 < cnt; g0 += SP_K) {
            const int4 q0 = *reinterpret_cast<const int4*>(&st_l[g0 + kq]);
            const int4 q1 = *reinterpret_cast<const int4*>(&st_l[g0 + kq + 4]);
            const int lk[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
            // byte offset of the lane's tap in slot g0 + kq + t, clamped onto the zeros
            const int oa = (g0 + kq) * WS * SA, ob = (g0 + kq) * WS * SB;
            const int ra = oa + (r + 1) * SA, rb = ob + (r + 1) * SB;
            const int ha = oa + (W + 1) * SA, hb = ob + (W + 1) * SB;
            const char* ca = reinterpret_cast<const char*>(st_a);
            const char* cb = reinterpret_cast<const char*>(st_b);
            v8u ah, al, brh, brl, bih, bil;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int ia = med3i(ra - (int)(short)(lk[t] & 0xFFFF), oa, ha);
              const int ib = med3i(rb - (lk[t] >> 16), ob, hb);
              const TA a = *reinterpret_cast<const TA*>(ca + ia + t * WS * SA);
              const TB b = *reinterpret_cast<const TB*>(cb + ib + t * WS * SB);
              if constexpr (PREC == 0) {
                ah[t] = (unsigned short)(a & 0xFFFFu);
                al[t] = (unsigned short)(a >> 16);
                brh[t] = (unsigned short)(b.x & 0xFFFFu);
                brl[t] = (unsigned short)(b.x >> 16);
                bih[t] = (unsigned short)(b.y & 0xFFFFu);
                bil[t] = (unsigned short)(b.y >> 16);
              } else {
                ah[t] = a;
                brh[t] = (unsigned short)(b & 0xFFFFu);
                bih[t] = (unsigned short)(b >> 16);
              }
            }
            cre = mfma16<PREC>(ah, brh, cre);
            cim = mfma16<PREC>(ah, bih, cim);
            if constexpr (PREC == 0) {
              cre = mfma16<PREC>(ah, brl, cre);
              cim = mfma16<PREC>(ah, bil, cim);
              cre = mfma16<PREC>(al, brh, cre);
              cim = mfma16<PREC>(al, bih, cim);
            }
          }
          __syncthreads();
        }
      }
    }
  }
  // accumulator v of lane: tile row 8 (v / 4) + 4 (lane / 32) + v % 4, column lane % 32
  float2* g = G + (size_t)sl * p.grid * p.grid;
  const int kx = (X0 + r) & (p.grid - 1);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    const int ky = (Y0 + row) & (p.grid - 1);
    g[(size_t)ky * p.grid + kx] = make_float2(cre[v], cim[v]);
  }
}

// Forward USFFT step (3): interpolate slab slab0 + (block % ns) of the grid
// at the samples whose wrapped base cell floor(X), floor(Y) lies in tile
// ring_tile(block / ns); the padded tile is staged in LDS.  Each sample has exactly
// one owner tile, so D is written once per sample.  The block's four waves
// take interleaved passes of 64 angles; a pass finds the m-interval of each
// angle that can own samples in the tile (the tile's own box), compacts
// the non-empty intervals over the wave's lanes, and walks the candidates
// 64 at a time, one per lane.
template <int M>
__global__ __launch_bounds__(NT) void k_interp(KParams p, const float2* __restrict__ G,
                                               void* __restrict__ D, int slab0, int tile, int ns) {
  constexpr int W = 2 * M;
  constexpr int PMAX = TILE_MAX + W - 1;
  constexpr int NW = NT / 64;
  __shared__ float2 st[PMAX * PMAX];
  const int P = tile + W - 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int sl = (int)(blockIdx.x % (unsigned)ns);  // slabs vary fastest, dense central tiles first
  const int l = slab0 + sl;
  const int ntx = p.grid / tile;
  int tx, ty;
  ring_tile((int)(blockIdx.x / (unsigned)ns), ntx, tx, ty);
  const int X0 = -(p.grid >> 1) + tx * tile;
  const int Y0 = -(p.grid >> 1) + ty * tile;
  const float gcl = p.gs * (float)l;
  const float e2b = __expf(-2.f * p.beta);
  const int half_m = (p.w_p >> 1) - 1;
  const size_t gbase = (size_t)sl * p.grid * p.grid;
  const float iP = 1.f / (float)P;
  // FFT_IO loads in flight per thread; a round's surplus lanes repeat the
  // last cell (same value, same LDS address), so no branch separates a load
  // from its store
  for (int e0 = threadIdx.x; e0 < P * P; e0 += NT * FFT_IO) {
    float2 v[FFT_IO];
    int ec[FFT_IO];
#pragma unroll
    for (int u = 0; u < FFT_IO; ++u) {
      ec[u] = min(e0 + u * NT, P * P - 1);
      const int yy = div24(ec[u], P, iP), xx = ec[u] - yy * P;
      const int ky = (Y0 - M + 1 + yy) & (p.grid - 1), kx = (X0 - M + 1 + xx) & (p.grid - 1);
      v[u] = G[gbase + (size_t)ky * p.grid + kx];
    }
#pragma unroll
    for (int u = 0; u < FFT_IO; ++u) st[ec[u]] = v[u];
  }
  __syncthreads();
  const float reach = sqrtf(0.25f * (float)p.grid * (float)p.grid + gcl * gcl) + 2.f;
  bool rx[3], ry[3];
#pragma unroll
  for (int s3 = 0; s3 < 3; ++s3) {
    const float x0 = (float)(X0 + (s3 - 1) * p.grid - 1), y0 = (float)(Y0 + (s3 - 1) * p.grid - 1);
    rx[s3] = x0 < reach && x0 + (float)(tile + 2) > -reach;
    ry[s3] = y0 < reach && y0 + (float)(tile + 2) > -reach;
  }
  for (int sy = -1; sy <= 1; ++sy) {
    if (!ry[sy + 1]) continue;
    for (int sx = -1; sx <= 1; ++sx) {
      if (!rx[sx + 1]) continue;
      const int ox = sx * p.grid + X0, oy = sy * p.grid + Y0;  // copy origin
      for (int th0 = wave * 64; th0 < p.n_theta; th0 += NW * 64) {
        const int th = th0 + lane;
        int mlo = 0, mhi = -1;
        const bool found =
            th < p.n_theta && tile_candidates(p.ncw, gcl, p.trig[th], (float)ox, (float)oy,
                                              (float)tile, (float)tile, half_m, mlo, mhi);
        const unsigned long long fm = __ballot(found);
        const int nseg = __popcll(fm);
        if (nseg == 0) continue;
        // compact: found lanes to 0 .. nseg-1 in lane order, the rest after
        const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
        const int dst = 4 * (found ? below : nseg + lane - below);
        const int len = __builtin_amdgcn_ds_permute(dst, found ? mhi - mlo + 1 : 0);
        const int smlo = __builtin_amdgcn_ds_permute(dst, mlo);
        const int sth = __builtin_amdgcn_ds_permute(dst, th);
        int incl = len;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int t = __shfl_up(incl, o);
          if (lane >= o) incl += t;
        }
        const int spre = incl - len;
        const int total = __shfl(incl, 63);
        int jcur = 0;
        for (int base = 0; base < total; base += 64) {
          const int i = base + lane;
          int j = jcur;
          for (int jj = jcur + 1; jj < nseg; ++jj) {
            const int s0 = __builtin_amdgcn_readlane(spre, jj);
            if (s0 > base + 63) break;
            if (s0 <= i) j = jj;
          }
          jcur = __builtin_amdgcn_readlane(j, 63);
          const int pj = __shfl(spre, j), mj = __shfl(smlo, j), tj = __shfl(sth, j);
          if (i >= total) continue;
          const int m = mj + (i - pj);
          float X, Y;
          sample_pos(p.ncw, gcl, p.trig[tj], m, X, Y);
          const float fXf = floorf(X), fYf = floorf(Y);
          const int bx = (int)fXf - ox;
          const int by = (int)fYf - oy;
          if (bx < 0 || bx >= tile || by < 0 || by >= tile) continue;  // not this tile's sample
          float wx[W], wy[W];
          gauss_taps<M>(X - fXf, p.beta, e2b, wx);
          gauss_taps<M>(Y - fYf, p.beta, e2b, wy);
          float2 acc = make_float2(0.f, 0.f);
#pragma unroll
          for (int jy = 0; jy < W; ++jy) {
            float2 row = make_float2(0.f, 0.f);
            const float2* src = st + (by + jy) * P + bx;
#pragma unroll
            for (int ix = 0; ix < W; ++ix) {
              row.x = fmaf(wx[ix], src[ix].x, row.x);
              row.y = fmaf(wx[ix], src[ix].y, row.y);
            }
            acc.x = fmaf(wy[jy], row.x, acc.x);
            acc.y = fmaf(wy[jy], row.y, acc.y);
          }
          st_c(D, ((size_t)l * p.n_theta + tj) * p.w_p + (m & (p.w_p - 1)),
               cscale(acc, p.fwd_D_scale), p.storage_dtype);
        }
      }
    }
  }
}

// ======================================================= slab 2D transforms
// Grid layout: G[slab_local][k2][k1], index k mod N_g.  After the row pass
// the first n entries of each row hold x1 = ix - n/2 (ix < n).

// Inverse FFT along x1 of each gridded slab row; the first n entries of
// the row then hold x1 = ix - n/2.
template <int LOGN>
__global__ __launch_bounds__(NTF) void k_grid_rows_inv(KParams p, float2* __restrict__ G,
                                                      int rows) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int N = p.grid;
  const int r0 = blockIdx.x * rows;
  float2* g = G + (size_t)blockIdx.y * N * N;
  stage_in<float2>(
      min(rows, N - r0) * N, [&](int e) { return g[(size_t)r0 * N + e]; },
      [&](int e, float2 v) { buf[e] = v; });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_grid, rows, p.tw, p.log2_twmax, true);
  const float2* res = buf;
  const float in = 1.f / (float)p.n;
  for (int e = threadIdx.x; e < rows * p.n; e += NTF) {
    const int b = div24(e, p.n, in), ix = e - b * p.n;
    if (r0 + b < N) g[(size_t)(r0 + b) * N + ix] = res[b * N + ((ix - p.n / 2) & (N - 1))];
  }
}

// k_grid_rows_inv for grid N = 64 R (512 or 1024) with one wave per row (wave_fft); each
// wave reads its whole row before writing the cropped n entries back.
template <int R>
__global__ __launch_bounds__(64 * WFFT_WAVES) void k_grid_rows_inv_w(KParams p, float2* __restrict__ G,
                                                                     int rows_per_wave) {
  constexpr int N = 64 * R;
  __shared__ float2 xch_all[WFFT_WAVES * wfft_xch(R)];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  float2* xch = xch_all + wv * wfft_xch(R);
  // 1024-point rows keep the first-stage twiddles in LDS (fewer registers, more waves)
  __shared__ float2 twa_s[R == 16 ? 15 * 64 : 1];
  float2* const twa = R == 16 ? twa_s : nullptr;
  WaveTw<R> t;
  wave_tw<R, R == 16>(p.tw, p.log2_twmax, true, t, twa);
  // slabs in reverse order: the gridding wrote the last ones last
  float2* g = G + (size_t)(gridDim.y - 1 - blockIdx.y) * N * N;
  const int r0 = (blockIdx.x * WFFT_WAVES + wv) * rows_per_wave;
  const int r1 = min(r0 + rows_per_wave, N);
  for (int row = r0; row < r1; ++row) {
    float2* gr = g + (size_t)row * N;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = gr[L + 64 * r];
    wave_fft<R, R == 16>(v, xch, t, true, twa);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int ix = (wave_out<R>(L, q) + p.n / 2) & (N - 1);  // entry (ix - n/2) mod N -> column ix
      if (ix < p.n) gr[ix] = v[q];
    }
  }
}

// g holds slabs g_l0 .. (all of them, or one streamed chunk).
template <int LOGN>
__global__ __launch_bounds__(NTF) void k_grid_cols_adj(KParams p, const float2* __restrict__ G,
                                                      void* __restrict__ g, int slab0, int cols,
                                                      int g_l0) {
  extern __shared__ float2 buf[];  // col_capacity(N) values (launch size)
  const int N = p.grid;
  const int ix0 = blockIdx.x * cols;
  const float icols = 1.f / (float)cols;
  const float2* gg = G + (size_t)blockIdx.y * N * N;
  stage_in<float2>(
      cols * N,
      [&](int e) {
        const int k2 = div24(e, cols, icols), c = e - k2 * cols;
        return (ix0 + c < p.n) ? gg[(size_t)k2 * N + ix0 + c] : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) {
        const int k2 = div24(e, cols, icols), c = e - k2 * cols;
        buf[c * N + k2] = v;
      });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_grid, cols, p.tw, p.log2_twmax, true);
  const float2* res = buf;
  const int l = slab0 + blockIdx.y;
  // four elements per thread at a time: their psi-correction loads are
  // issued together (unconditionally, clamped), the stores follow
  const int total = cols * p.n;
  with_storage(p.storage_dtype, [&](auto ty) {
    for (int e0 = threadIdx.x; e0 < total; e0 += 4 * NTF) {
      float2 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * NTF, total - 1);
        const int y = div24(e, cols, icols), c = e - y * cols;
        const float dp = p.deapod[min(ix0 + c, p.n - 1)] * p.deapod[y];
        v[u] = cscale(res[c * N + ((y - p.n / 2) & (N - 1))], dp);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * NTF;
        const int y = div24(e, cols, icols), c = e - y * cols;
        if (e < total && ix0 + c < p.n)
          st_ct<decltype(ty)::value>(g, ((size_t)(l - g_l0) * p.n + y) * p.n + ix0 + c, v[u]);
      }
    }
  });
}

// k_grid_cols_adj for grid N = 64 R (512 or 1024) with one wave per column: a block stages CW
// columns of the row-transformed slab (rows of CW consecutive entries) into
// LDS column-major with stride wcol_stride(R, CW), each wave transforms CW / 8
// of them in place and writes the cropped column back, and the block writes
// rows y of the slab plane, CW consecutive columns per row, with the psi
// correction.
template <int R, int CW>
__global__ __launch_bounds__(512) void k_grid_cols_adj_w(KParams p, const float2* __restrict__ G,
                                                         void* __restrict__ g, int slab0, int g_l0) {
  constexpr int N = 64 * R;
  constexpr int S = wcol_stride(R, CW);
  __shared__ float2 buf[CW * S];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int ix0 = blockIdx.x * CW;
  const float2* gg = G + (size_t)blockIdx.y * N * N;
  // the block's whole input in one round of loads (2 x 8 per thread at
  // N = 512, CW = 16)
  stage_in<float2, N * CW / 512 < 16 ? N * CW / 512 : 16>(
      N * CW,
      [&](int e) {
        const int k2 = e / CW, c = e % CW;
        const float2 v = gg[(size_t)k2 * N + min(ix0 + c, p.n - 1)];
        return ix0 + c < p.n ? v : make_float2(0.f, 0.f);
      },
      [&](int e, float2 v) { buf[(e % CW) * S + e / CW] = v; });
  WaveTw<R> t;
  wave_tw<R>(p.tw, p.log2_twmax, true, t);
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < CW / 8; ++cc) {
    float2* col = buf + (wv * (CW / 8) + cc) * S;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = col[L + 64 * r];
    wave_fft<R>(v, col, t, true);
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int y = (wave_out<R>(L, q) + p.n / 2) & (N - 1);  // entry (y - n/2) mod N -> row y
      if (y < p.n) col[y] = v[q];
    }
  }
  __syncthreads();
  const int l = slab0 + blockIdx.y;
  // each thread keeps one column and takes every (512 / CW)-th row
  static_assert(512 % CW == 0, "a thread's column must not change between rows");
  const int c = threadIdx.x % CW, ix = ix0 + c;
  if (ix >= p.n) return;
  const float dx = p.deapod[ix];
  with_storage(p.storage_dtype, [&](auto ty) {
#pragma unroll 8
    for (int y = threadIdx.x / CW; y < p.n; y += 512 / CW) {
      const float2 v = cscale(buf[c * S + y], dx * p.deapod[y]);
      st_ct<decltype(ty)::value>(g, ((size_t)(l - g_l0) * p.n + y) * p.n + ix, v);
    }
  });
}

template <int LOGN>
__global__ __launch_bounds__(NTF) void k_grid_cols_fwd(KParams p, const void* __restrict__ g,
                                                      float2* __restrict__ G, int slab0, int cols) {
  extern __shared__ float2 buf[];  // col_capacity(N) values (launch size)
  const int N = p.grid;
  const int ix0 = blockIdx.x * cols;
  const float icols = 1.f / (float)cols;
  const int l = slab0 + blockIdx.y;
  lds_zero(buf, cols * N);
  __syncthreads();
  with_storage(p.storage_dtype, [&](auto ty) {
    stage_in<float2>(
        cols * p.n,
        [&](int e) {
          // psi correction with the value's own loads (a select of a loaded
          // value, or a load at the placing step, would be waited for at once)
          const int y = div24(e, cols, icols), ix = ix0 + e - y * cols;
          const int ixc = min(ix, p.n - 1);
          const float2 v = ld_ct<decltype(ty)::value>(g, ((size_t)l * p.n + y) * p.n + ixc);
          const float dp = p.deapod[ixc] * p.deapod[y];
          return cscale(v, ix < p.n ? dp : 0.f);
        },
        [&](int e, float2 v) {
          const int y = div24(e, cols, icols), c = e - y * cols;
          if (ix0 + c < p.n) buf[c * N + ((y - p.n / 2) & (N - 1))] = v;
        });
  });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_grid, cols, p.tw, p.log2_twmax, false);
  const float2* res = buf;
  float2* gg = G + (size_t)blockIdx.y * N * N;
  for (int e = threadIdx.x; e < cols * N; e += NTF) {
    const int k2 = div24(e, cols, icols), c = e - k2 * cols;
    if (ix0 + c < p.n) gg[(size_t)k2 * N + ix0 + c] = res[c * N + k2];
  }
}

template <int LOGN>
__global__ __launch_bounds__(NTF) void k_grid_rows_fwd(KParams p, float2* __restrict__ G,
                                                      int rows) {
  extern __shared__ float2 buf[];  // fft_capacity(N) values (launch size)
  const int N = p.grid;
  const int r0 = blockIdx.x * rows;
  float2* g = G + (size_t)blockIdx.y * N * N;
  const float in = 1.f / (float)p.n;
  lds_zero(buf, rows * N);
  __syncthreads();
  stage_in<float2>(
      min(rows, N - r0) * p.n,
      [&](int e) {
        const int b = div24(e, p.n, in), ix = e - b * p.n;
        return g[(size_t)(r0 + b) * N + ix];
      },
      [&](int e, float2 v) {
        const int b = div24(e, p.n, in), ix = e - b * p.n;
        buf[b * N + ((ix - p.n / 2) & (N - 1))] = v;
      });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_grid, rows, p.tw, p.log2_twmax, false);
  const float2* res = buf;
  for (int e = threadIdx.x; e < rows * N; e += NTF) {
    const int b = e >> p.log2_grid;
    if (r0 + b < N) g[(size_t)(r0 + b) * N + (e & (N - 1))] = res[e];
  }
}

// k_grid_cols_fwd for grid N = 64 R (512 or 1024) with one wave per column: CW columns of the
// slab plane (psi-corrected) are placed at rows (y - n/2) mod N of LDS
// columns, transformed in place (entries that hold no row are zeroed on
// loading), and written as rows k2 of CW consecutive grid columns.
template <int R, int CW>
__global__ __launch_bounds__(512) void k_grid_cols_fwd_w(KParams p, const void* __restrict__ g,
                                                         float2* __restrict__ G, int slab0) {
  constexpr int N = 64 * R;
  constexpr int S = wcol_stride(R, CW);
  __shared__ float2 buf[CW * S];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  const int ix0 = blockIdx.x * CW;
  const int l = slab0 + blockIdx.y;
  with_storage(p.storage_dtype, [&](auto ty) {
    stage_in<float2>(
        p.n * CW,
        [&](int e) {
          // psi correction with the value's own loads (a select of a loaded
          // value, or a load at the placing step, would be waited for at once)
          const int y = e / CW, ix = ix0 + e % CW;
          const int ixc = min(ix, p.n - 1);
          const float2 v = ld_ct<decltype(ty)::value>(g, ((size_t)l * p.n + y) * p.n + ixc);
          const float dp = p.deapod[ixc] * p.deapod[y];
          return cscale(v, ix < p.n ? dp : 0.f);
        },
        [&](int e, float2 v) { buf[(e % CW) * S + (((e / CW) - p.n / 2) & (N - 1))] = v; });
  });
  WaveTw<R> t;
  wave_tw<R>(p.tw, p.log2_twmax, false, t);
  __syncthreads();
#pragma unroll
  for (int cc = 0; cc < CW / 8; ++cc) {
    float2* col = buf + (wv * (CW / 8) + cc) * S;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int pos = L + 64 * r;  // entry (y - n/2) mod N holds row y
      v[r] = ((pos + p.n / 2) & (N - 1)) < p.n ? col[pos] : make_float2(0.f, 0.f);
    }
    wave_fft<R>(v, col, t, false);
#pragma unroll
    for (int q = 0; q < R; ++q) col[wave_out<R>(L, q)] = v[q];
  }
  __syncthreads();
  float2* gg = G + (size_t)blockIdx.y * N * N;
  for (int e = threadIdx.x; e < N * CW; e += 512) {
    const int k2 = e / CW, c = e % CW;
    if (ix0 + c < p.n) gg[(size_t)k2 * N + ix0 + c] = buf[c * S + k2];
  }
}

// k_grid_rows_fwd for grid N = 64 R (512 or 1024) with one wave per row: the row's n entries
// are loaded at (ix - n/2) mod N (zero elsewhere), transformed, and the
// whole row is written back.
template <int R>
__global__ __launch_bounds__(64 * WFFT_WAVES) void k_grid_rows_fwd_w(KParams p, float2* __restrict__ G,
                                                                     int rows_per_wave) {
  constexpr int N = 64 * R;
  __shared__ float2 xch_all[WFFT_WAVES * wfft_xch(R)];
  const int wv = threadIdx.x >> 6, L = threadIdx.x & 63;
  float2* xch = xch_all + wv * wfft_xch(R);
  // 1024-point rows keep the first-stage twiddles in LDS (fewer registers, more waves)
  __shared__ float2 twa_s[R == 16 ? 15 * 64 : 1];
  float2* const twa = R == 16 ? twa_s : nullptr;
  WaveTw<R> t;
  wave_tw<R, R == 16>(p.tw, p.log2_twmax, false, t, twa);
  // slabs in reverse order: the column pass wrote the last ones last
  float2* g = G + (size_t)(gridDim.y - 1 - blockIdx.y) * N * N;
  const int r0 = (blockIdx.x * WFFT_WAVES + wv) * rows_per_wave;
  const int r1 = min(r0 + rows_per_wave, N);
  for (int row = r0; row < r1; ++row) {
    float2* gr = g + (size_t)row * N;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int ix = (L + 64 * r + p.n / 2) & (N - 1);  // entry (ix - n/2) mod N holds column ix
      v[r] = ix < p.n ? gr[ix] : make_float2(0.f, 0.f);
    }
    wave_fft<R, R == 16>(v, xch, t, false, twa);
#pragma unroll
    for (int q = 0; q < R; ++q) gr[wave_out<R>(L, q)] = v[q];
  }
}

// ============================================================ x3 transform
// Both directions are real matrix products on the matrix cores, with the
// phase tables split on the host into 16-bit hi + lo parts:
//   adj: vol[z][col] = sum_k A[z][k] B[k][col], k = 2l + c,
//        B[2l][col] = Re g[l][col], B[2l + 1][col] = Im g[l][col];
//   fwd: G[2l + c][col] = sum_z A[2l + c][z] f[z][col] gives Re / Im ghat.
// Lane l of a 32 x 32 x 16 product (v_mfma_f32_32x32x16) holds
// A[l % 32][8 (l / 32) + t], B[8 (l / 32) + t][l % 32] and
// C[8 (v / 4) + 4 (l / 32) + v % 4][l % 32].  Float32 operands are split into
// bf16 hi + lo (three products); float16 / bfloat16 slab data are exact in
// their own format (two products).

__device__ __forceinline__ void split8(const float x[8], v8u& hi, v8u& lo) {
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
  v4u h4, l4;
#pragma unroll
  for (int t = 0; t < 8; t += 2) {
    const unsigned hh = bf16_pair(x[t], x[t + 1]);
    h4[t >> 1] = hh;
    l4[t >> 1] = bf16_pair(x[t] - __uint_as_float(hh << 16), x[t + 1] - __uint_as_float(hh & 0xFFFF0000u));
  }
  hi = __builtin_bit_cast(v8u, h4);
  lo = __builtin_bit_cast(v8u, l4);
}

// Raw B operand of K-step k0 for the adjoint: this lane's slabs
// (k0 / 2 + 4 h .. + 3) of column `cidx`, float2 (PREC 0) or 16-bit pairs.
template <int PREC>
struct X3AdjB {
  typedef typename std::conditional<PREC == 0, float2, unsigned>::type T;
  T v[4];
};
template <int PREC>
__device__ __forceinline__ void x3_adj_loadb(const KParams& p, const void* g, int ncol, bool cok,
                                             size_t cidx, int k0, int h, X3AdjB<PREC>& b) {
  const int l0 = (k0 >> 1) + 4 * h;
  // loads from clamped indices are unconditional (no branches around them);
  // out-of-range values are replaced afterwards
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int l = l0 + q;
    const bool ok = cok && l < p.n_slab;
    const size_t i = (size_t)min(l, p.n_slab - 1) * ncol + cidx;
    if constexpr (PREC == 0) {
      const float2 v = reinterpret_cast<const float2*>(g)[i];
      b.v[q] = ok ? v : make_float2(0.f, 0.f);
    } else {
      const unsigned v = reinterpret_cast<const unsigned*>(g)[i];
      b.v[q] = ok ? v : 0u;
    }
  }
}

// vol[z0 - out_z0 + z][col0 + col] for z in [0, nzc) and the ncol columns
// col of g (slab stride g_ld columns); vol rows have v_ld columns.  Each
// slab-plane value is read once: a wave owns 32 columns and ZT 32-row z
// tiles (ZT = 8: accumulators for 256 slices; 2 for z chunks of at most 64
// slices), the block's four waves take neighbouring column tiles, and the
// phase-table fragments of the block's rows are staged once per K step in
// LDS (double buffered; the next step's fragments are fetched from HBM
// while the current step's products run).  blockIdx.y selects row blocks.
constexpr int X3B_WAVES = 4;
constexpr int X3B_ZT = 8;
constexpr int X3B_ROWS = 32 * X3B_ZT;  // slices per block

template <int PREC, int ZT>
__global__ __launch_bounds__(64 * X3B_WAVES) __attribute__((amdgpu_waves_per_eu(2))) void k_x3_adj_b(KParams p, const void* __restrict__ g,
                                                             int g_ld, float* __restrict__ vol,
                                                             int v_ld, int col0, int ncol, int z0,
                                                             int nzc, int out_z0) {
  // [buffer][hi, lo][row * 2 + half]: the fragments of one K step
  constexpr int ROWS = 32 * ZT;  // slices per block
  __shared__ v8u sa[2][2][ROWS * 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int col = (blockIdx.x * X3B_WAVES + wave) * 32 + r;
  const int zb = blockIdx.y * ROWS;
  const float outs = p.x3_out_scale * (p.dyn ? p.dyn[1] : 1.f);
  const int K = p.x3a_k;
  const bool cok = col < ncol;
  const size_t cidx = cok ? col : 0;
  // this thread's share of a step's fragments: 4 of the 2 x 512
  // this thread's share of a step's fragments: 2 x 2 ROWS of them
  constexpr int NA = (4 * ROWS) / (64 * X3B_WAVES);
  v8u an[NA];
  auto fetch_a = [&](int st) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int i = threadIdx.x + 64 * X3B_WAVES * u;
      const int hl = i / (2 * ROWS), f = i % (2 * ROWS);
      const int row = min(z0 + zb + (f >> 1), p.x3a_rows - 1);
      const size_t o = (((size_t)st * p.x3a_rows + row) * 2 + (f & 1)) * 8 + (hl ? (size_t)p.x3a_rows * K : 0);
      an[u] = *reinterpret_cast<const v8u*>(p.x3a + o);
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < NA; ++u) {
      const int i = threadIdx.x + 64 * X3B_WAVES * u;
      sa[buf][i / (2 * ROWS)][i % (2 * ROWS)] = an[u];
    }
  };
  v16f acc[ZT] = {};
  X3AdjB<PREC> bc, bn;
  x3_adj_loadb<PREC>(p, g, g_ld, cok, cidx, 0, h, bc);
  fetch_a(0);
  store_a(0);
  const int ns = K >> 4;
  for (int st = 0; st < ns; ++st) {
    __syncthreads();  // step st's fragments are in LDS; step st - 1's buffer is free
    const int nx = min(st + 1, ns - 1);  // the last step refetches itself
    x3_adj_loadb<PREC>(p, g, g_ld, cok, cidx, nx << 4, h, bn);
    fetch_a(nx);
    v8u bh, bl;
    if constexpr (PREC == 0) {
      float x[8];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[2 * q] = bc.v[q].x;
        x[2 * q + 1] = bc.v[q].y;
      }
      split8(x, bh, bl);
    } else {
      // 16-bit complex pairs (re | im << 16) are the operand's pairs of k
      bh = __builtin_bit_cast(v8u, make_uint4(bc.v[0], bc.v[1], bc.v[2], bc.v[3]));
    }
    const v8u* ah = sa[st & 1][0];
    const v8u* al = sa[st & 1][1];
#pragma unroll
    for (int i = 0; i < ZT; ++i) {
      const int f = (32 * i + r) * 2 + h;
      acc[i] = mfma16<PREC>(ah[f], bh, acc[i]);
      acc[i] = mfma16<PREC>(al[f], bh, acc[i]);
      if constexpr (PREC == 0) acc[i] = mfma16<0>(ah[f], bl, acc[i]);
    }
    if (st + 1 < ns) store_a((st + 1) & 1);
    bc = bn;
  }
  if (!cok) return;
#pragma unroll
  for (int i = 0; i < ZT; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int z = zb + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
      if (z < nzc) vol[(size_t)(z0 - out_z0 + z) * v_ld + col0 + col] = acc[i][v] * outs;
    }
}


// ghat[l][col] = sum_z exp(-2 pi i x3 l cos(phi) / h_p) f[z][col], each
// volume value read once per 256 rows: a wave owns 32 columns and X3B_ZT
// 32-row tiles of the 2 n_slab rows, the block's waves take neighbouring
// column tiles, and the phase fragments of the block's rows are staged per
// K step in double-buffered LDS (as in k_x3_adj_b).
__global__ __launch_bounds__(64 * X3B_WAVES) __attribute__((amdgpu_waves_per_eu(2))) void k_x3_fwd_b(
    KParams p, const float* __restrict__ f, void* __restrict__ g) {
  __shared__ v8u sa[2][2][X3B_ROWS * 2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r = lane & 31, h = lane >> 5;
  const int ncol = p.n * p.n;
  const int col = (blockIdx.x * X3B_WAVES + wave) * 32 + r;
  const int mb = blockIdx.y * X3B_ROWS;  // rows 2l + c
  const int K = p.x3f_k;
  const bool cok = col < ncol;
  const size_t cidx = cok ? col : 0;
  v8u an[4];
  auto fetch_a = [&](int st) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + 64 * X3B_WAVES * u;
      const int hl = i >> 9, fr = i & 511;
      const int row = min(mb + (fr >> 1), p.x3f_rows - 1);
      const size_t o = (((size_t)st * p.x3f_rows + row) * 2 + (fr & 1)) * 8 + (hl ? (size_t)p.x3f_rows * K : 0);
      an[u] = *reinterpret_cast<const v8u*>(p.x3f + o);
    }
  };
  auto store_a = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + 64 * X3B_WAVES * u;
      sa[buf][i >> 9][i & 511] = an[u];
    }
  };
  auto load_b = [&](int st, float x[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int z = 16 * st + 8 * h + t;
      x[t] = f[(size_t)min(z, p.nz - 1) * ncol + cidx];
      if (!cok || z >= p.nz) x[t] = 0.f;
    }
  };
  v16f acc[X3B_ZT] = {};
  float xc[8], xn[8];
  load_b(0, xc);
  fetch_a(0);
  store_a(0);
  const int ns = K >> 4;
  for (int st = 0; st < ns; ++st) {
    __syncthreads();
    const int nx = min(st + 1, ns - 1);
    load_b(nx, xn);
    fetch_a(nx);
    v8u bh, bl;
    split8(xc, bh, bl);
    const v8u* ah = sa[st & 1][0];
    const v8u* al = sa[st & 1][1];
#pragma unroll
    for (int i = 0; i < X3B_ZT; ++i) {
      const int fr = (32 * i + r) * 2 + h;
      acc[i] = mfma16<0>(ah[fr], bh, acc[i]);
      acc[i] = mfma16<0>(ah[fr], bl, acc[i]);
      acc[i] = mfma16<0>(al[fr], bh, acc[i]);
    }
    if (st + 1 < ns) store_a((st + 1) & 1);
#pragma unroll
    for (int t = 0; t < 8; ++t) xc[t] = xn[t];
  }
  if (!cok) return;
  const float gs = p.fwd_g_scale * (p.dyn ? p.dyn[0] : 1.f);
#pragma unroll
  for (int i = 0; i < X3B_ZT; ++i)
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
      const int m = mb + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
      const int l = m >> 1;
      if (l < p.n_slab)
        st_c(g, (size_t)l * ncol + col, make_float2(acc[i][v] * gs, acc[i][v + 1] * gs),
             p.storage_dtype);
    }
}

// Float16 storage: the call's input is scaled by f = 2^-e so that its largest
// magnitude lies in [0.5, 1), which keeps the stored spectra and slab planes
// inside the float16 range for any input scale.  Block maxima first, then
// one block forms f and 1/f (exact powers of two) in dyn[0], dyn[1].
constexpr int ABSMAX_BLOCKS = 1024;

// largest magnitude among the elements of one 16-byte chunk
template <int DT>
__device__ __forceinline__ float absmax16(uint4 v) {
  const unsigned w[4] = {v.x, v.y, v.z, v.w};
  float m = 0.f;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if constexpr (DT == LAMINO_F32) {
      m = fmaxf(m, fabsf(__uint_as_float(w[k])));
    } else if constexpr (DT == LAMINO_BF16) {
      m = fmaxf(m, fmaxf(fabsf(__uint_as_float(w[k] << 16)), fabsf(__uint_as_float(w[k] & 0xFFFF0000u))));
    } else if constexpr (DT == LAMINO_F16) {
      const float a = __half2float(__ushort_as_half((unsigned short)(w[k] & 0xFFFFu)));
      const float b = __half2float(__ushort_as_half((unsigned short)(w[k] >> 16)));
      m = fmaxf(m, fmaxf(fabsf(a), fabsf(b)));
    } else if constexpr (DT == LAMINO_U16) {
      m = fmaxf(m, (float)max(w[k] & 0xFFFFu, w[k] >> 16));
    } else {
      const unsigned b = max(max(w[k] & 0xFFu, (w[k] >> 8) & 0xFFu), max((w[k] >> 16) & 0xFFu, w[k] >> 24));
      m = fmaxf(m, (float)b);
    }
  }
  return m;
}

// 16-byte loads (four in flight per thread) when the input is 16-byte
// aligned, element loads for the rest
template <int DT>
// accumulate != 0: each block keeps the larger of its new maximum and the
// value already in part[blockIdx.x] (inputs scanned chunk by chunk)
__global__ __launch_bounds__(256) void k_absmax_partial(const void* __restrict__ x, size_t n,
                                                         float* __restrict__ part, int accumulate) {
  constexpr size_t PER = DT == LAMINO_F32 ? 4 : (DT == LAMINO_U8 ? 16 : 8);  // elements per chunk
  __shared__ float red[4];
  float m = 0.f;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t nv = 0;
  if ((reinterpret_cast<uintptr_t>(x) & 15) == 0) {
    nv = n / PER;
    const uint4* v = reinterpret_cast<const uint4*>(x);
    size_t i = tid;
    for (; i + 3 * stride < nv; i += 4 * stride) {
      const uint4 a = v[i], b = v[i + stride], c = v[i + 2 * stride], d = v[i + 3 * stride];
      m = fmaxf(m, fmaxf(fmaxf(absmax16<DT>(a), absmax16<DT>(b)), fmaxf(absmax16<DT>(c), absmax16<DT>(d))));
    }
    for (; i < nv; i += stride) m = fmaxf(m, absmax16<DT>(v[i]));
  }
  for (size_t i = nv * PER + tid; i < n; i += stride) m = fmaxf(m, fabsf(ld_r(x, i, DT)));
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float mb = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    part[blockIdx.x] = accumulate ? fmaxf(mb, part[blockIdx.x]) : mb;
  }
}

// nb partial maxima (0: none) and a host-known bound `extra`
__global__ __launch_bounds__(256) void k_absmax_final(float* __restrict__ dyn, int nb, float extra) {
  __shared__ float red[4];
  float m = threadIdx.x == 0 ? extra : 0.f;
  for (int i = threadIdx.x; i < nb; i += 256) m = fmaxf(m, dyn[2 + i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    int e = 0;
    if (m > 0.f && isfinite(m)) frexpf(m, &e);  // m = frac 2^e, frac in [0.5, 1)
    dyn[0] = ldexpf(1.f, -e);
    dyn[1] = ldexpf(1.f, e);
  }
}

// ================================================================ drivers
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }
// Complex values per block of the block slab-column kernels: from 2048
// points on the block holds the largest buffer (LDS_CPLX_MAX: 4, 2 or 1
// columns), so that it reads 32-byte rather than 16-byte row segments at 2048
// points (slab stage of the N = 1024 FBP 40.1 -> 35.9 ms).  The detector
// column kernels keep fft_capacity (wider blocks were slower there).
static inline int col_capacity(int N) { return N >= 2048 ? LDS_CPLX_MAX : fft_capacity(N); }

// The instantiation of an FFT kernel for transforms of N points: a fixed
// size from 256 to 8192 points (8192: the wide passes), else the run-time one.
#define FFT_KERNEL(k, N)                                                                  \
  ((N) == 512 ? k<9> : (N) == 256 ? k<8> : (N) == 1024 ? k<10> : (N) == 2048 ? k<11>   \
   : (N) == 4096 ? k<12> : (N) == 8192 ? k<13> : k<0>)

// Sets the float16 input factor of a call from its input (x != NULL) or from
// a known bound alone.
// Block maxima of x[0 .. n) into dyn[2 ..] (nb blocks); with accumulate the
// maxima of earlier chunks are kept (nb must then be the same for every chunk).
static void absmax_partial(const KParams& kp, const void* x, size_t n, int dt, int nb,
                           int accumulate, hipStream_t s) {
  float* part = const_cast<float*>(kp.dyn) + 2;
  switch (dt) {
    case LAMINO_F32: hipLaunchKernelGGL(k_absmax_partial<LAMINO_F32>, dim3(nb), dim3(256), 0, s, x, n, part, accumulate); break;
    case LAMINO_F16: hipLaunchKernelGGL(k_absmax_partial<LAMINO_F16>, dim3(nb), dim3(256), 0, s, x, n, part, accumulate); break;
    case LAMINO_BF16: hipLaunchKernelGGL(k_absmax_partial<LAMINO_BF16>, dim3(nb), dim3(256), 0, s, x, n, part, accumulate); break;
    case LAMINO_U8: hipLaunchKernelGGL(k_absmax_partial<LAMINO_U8>, dim3(nb), dim3(256), 0, s, x, n, part, accumulate); break;
    default: hipLaunchKernelGGL(k_absmax_partial<LAMINO_U16>, dim3(nb), dim3(256), 0, s, x, n, part, accumulate); break;
  }
}

// Sets the float16 input factor of a call from its input (x != NULL) or from
// a known bound alone.
static void input_factor(const KParams& kp, const void* x, size_t n, int dt, float bound,
                         hipStream_t s) {
  float* dyn = const_cast<float*>(kp.dyn);
  int nb = 0;
  if (x) {
    nb = (int)std::min<size_t>(ABSMAX_BLOCKS, std::max<size_t>(1, (n + 255) / 256));
    absmax_partial(kp, x, n, dt, nb, 0, s);
  }
  hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, s, dyn, nb, bound);
}

static int spread_tile(const KParams& p) { return p.grid <= 128 ? (p.grid < 32 ? p.grid : 32) : 64; }

// Gridding launches are one-dimensional (block = slab + ns * tile rank) and
// hold at most GRID_BLOCKS_MAX blocks: larger slab chunks go in several
// launches of fewer slabs (grid 8192 has 65536 spreading tiles per slab).
constexpr int GRID_BLOCKS_MAX = 1 << 22;

// D holds slabs d_l0 .. (all of them, or one streamed chunk); G the planes
// of slabs s0 .. s0 + ns - 1
template <int M>
static void launch_spread(const KParams& kp, const void* D, float2* G, int s0, int ns, int d_l0,
                          hipStream_t s) {
  const int tiles = (kp.grid / SP_T) * (kp.grid / SP_T);
  const int per = std::max(1, std::min(ns, GRID_BLOCKS_MAX / tiles));
  for (int j = 0; j < ns; j += per) {
    const int nj = std::min(per, ns - j);
    float2* Gj = G + (size_t)j * kp.grid * kp.grid;
    const dim3 grid((unsigned)nj * (unsigned)tiles);
    if (kp.storage_dtype == LAMINO_F32)
      hipLaunchKernelGGL((k_spread<M, 0>), grid, dim3(64), 0, s, kp, D, Gj, s0 + j, d_l0, nj);
    else if (kp.storage_dtype == LAMINO_F16)
      hipLaunchKernelGGL((k_spread<M, 1>), grid, dim3(64), 0, s, kp, D, Gj, s0 + j, d_l0, nj);
    else
      hipLaunchKernelGGL((k_spread<M, 2>), grid, dim3(64), 0, s, kp, D, Gj, s0 + j, d_l0, nj);
  }
}
template <int M>
static void launch_interp(const KParams& kp, const float2* G, void* D, int s0, int ns, int tile,
                          hipStream_t s) {
  const int tiles = (kp.grid / tile) * (kp.grid / tile);
  const int per = std::max(1, std::min(ns, GRID_BLOCKS_MAX / tiles));
  for (int j = 0; j < ns; j += per) {
    const int nj = std::min(per, ns - j);
    hipLaunchKernelGGL(k_interp<M>, dim3((unsigned)nj * (unsigned)tiles), dim3(NT), 0, s, kp,
                       G + (size_t)j * kp.grid * kp.grid, D, s0 + j, tile, nj);
  }
}

static void spread_dispatch(const KParams& kp, const void* D, float2* G, int s0, int ns, int d_l0,
                            hipStream_t s) {
  switch (kp.M) {
    case 2: launch_spread<2>(kp, D, G, s0, ns, d_l0, s); break;
    case 3: launch_spread<3>(kp, D, G, s0, ns, d_l0, s); break;
    case 4: launch_spread<4>(kp, D, G, s0, ns, d_l0, s); break;
    case 5: launch_spread<5>(kp, D, G, s0, ns, d_l0, s); break;
    case 6: launch_spread<6>(kp, D, G, s0, ns, d_l0, s); break;
    case 7: launch_spread<7>(kp, D, G, s0, ns, d_l0, s); break;
    default: launch_spread<8>(kp, D, G, s0, ns, d_l0, s); break;
  }
}
static void interp_dispatch(const KParams& kp, const float2* G, void* D, int s0, int ns,
                            hipStream_t s) {
  const int tile = spread_tile(kp);
  switch (kp.M) {
    case 2: launch_interp<2>(kp, G, D, s0, ns, tile, s); break;
    case 3: launch_interp<3>(kp, G, D, s0, ns, tile, s); break;
    case 4: launch_interp<4>(kp, G, D, s0, ns, tile, s); break;
    case 5: launch_interp<5>(kp, G, D, s0, ns, tile, s); break;
    case 6: launch_interp<6>(kp, G, D, s0, ns, tile, s); break;
    case 7: launch_interp<7>(kp, G, D, s0, ns, tile, s); break;
    default: launch_interp<8>(kp, G, D, s0, ns, tile, s); break;
  }
}

static inline char* wptr(const lamino_plan_s* p, size_t off) {
  return static_cast<char*>(p->d_work) + off;
}

// x3 transform of the columns [col0, col0 + ncol) of the slabs in g (slab
// stride g_ld columns): vol[z - out_z0][vcol0 + col] for z in [z0, z0 + nzc),
// vol rows of v_ld columns.
static void launch_x3_adj(const KParams& kp, const void* g, int g_ld, float* vol, int v_ld,
                          int vcol0, int ncol, int z0, int nzc, int out_z0, hipStream_t s) {
  // z chunks of up to 64 slices take blocks of 64 rows (two accumulator
  // tiles per wave), longer ones blocks of 256
  const bool narrow = nzc <= 64;
  const dim3 grid(cdiv(ncol, 32 * X3B_WAVES), cdiv(nzc, narrow ? 64 : 32 * X3B_ZT));
  const dim3 blk(64 * X3B_WAVES);
#define X3ADJ(P) (narrow ? k_x3_adj_b<P, 2> : k_x3_adj_b<P, X3B_ZT>)
  if (kp.storage_dtype == LAMINO_F32)
    hipLaunchKernelGGL(X3ADJ(0), grid, blk, 0, s, kp, g, g_ld, vol, v_ld, vcol0, ncol, z0, nzc, out_z0);
  else if (kp.storage_dtype == LAMINO_F16)
    hipLaunchKernelGGL(X3ADJ(1), grid, blk, 0, s, kp, g, g_ld, vol, v_ld, vcol0, ncol, z0, nzc, out_z0);
  else
    hipLaunchKernelGGL(X3ADJ(2), grid, blk, 0, s, kp, g, g_ld, vol, v_ld, vcol0, ncol, z0, nzc, out_z0);
#undef X3ADJ
}

// Backprojection pipeline.  Device-resident plans with device data and
// volume run every stage on `s` in order.  Otherwise (host data or volume,
// spectra or slab planes in host memory) the chunks move between host and
// device on the plan's copy streams: s_in brings chunks in, s_out takes
// results out, each through two alternating buffers, and events order
//   copy-in of chunk c  after  the kernels of chunk c - 2 released its buffer,
//   kernels of chunk c  after  its copy-in and after the copy-out of chunk
//                              c - 2 released the output buffer,
//   copy-out of chunk c after  the kernels of chunk c.
// Events 0-1: copy-in done, 2-3: input buffer released, 4-5: kernels done,
// 6-7: copy-out done (index = chunk parity); 8-9: stream joins.
hipError_t run_backprojection(const lamino_plan_s* p, const void* d_data, float* d_vol,
                              bool fbp_filter, hipStream_t s, const BackprojOpts& o) {
  KParams kp = make_params(p, fbp_filter, o.tables, o.work);
  char* const work = static_cast<char*>(o.work ? o.work : p->d_work);
  char* const io = static_cast<char*>(o.io);
  char* const hsp = static_cast<char*>(p->h_spill);
  const bool timing = o.timing;
  const bool host_in = o.h_data != nullptr, host_out = o.h_vol != nullptr;
  const bool piped = host_in || host_out || p->spill_D || p->spill_g;
  lamino_plan_s* pm = const_cast<lamino_plan_s*>(p);
  hipStream_t si = nullptr, so = nullptr;
  hipEvent_t* ev = pm->ev;
  if (piped) {
    const hipError_t e = ensure_pipe(pm);
    if (e != hipSuccess) return e;
    si = p->s_in;
    so = p->s_out;
    // every event starts complete at this point of s, and the copy streams
    // start after the work already on s
    for (int i = 0; i < 10; ++i) (void)hipEventRecord(ev[i], s);
    (void)hipStreamWaitEvent(si, ev[8], 0);
    (void)hipStreamWaitEvent(so, ev[8], 0);
  }
  auto rec = [&](int i, hipStream_t st) { (void)hipEventRecord(ev[i], st); };
  auto wait = [&](hipStream_t st, int i) { (void)hipStreamWaitEvent(st, ev[i], 0); };
  const size_t sb = storage_bytes(p->opts.storage_dtype);
  const size_t db = data_bytes(p->opts.data_dtype);
  const size_t ncol = (size_t)p->n * p->n;
  const size_t proj = (size_t)p->h * p->w;  // elements per projection
  kp.dark = o.dark;
  kp.flat = o.flat;
  kp.min_ratio = o.min_ratio;
  if (kp.dyn) {
    if (o.dark) {
      // raw counts: the corrected values are bounded by -log(min_ratio)
      input_factor(kp, nullptr, 0, 0, -std::log(o.min_ratio), s);
    } else if (!host_in) {
      input_factor(kp, d_data, (size_t)p->n_theta * proj, p->opts.data_dtype, 0.f, s);
    } else {
      // host data: one scan pass over the projection chunks, maxima kept per block
      for (int t0 = 0, c = 0; t0 < p->n_theta; t0 += p->theta_chunk, ++c) {
        const int nt = std::min(p->theta_chunk, p->n_theta - t0);
        char* buf = io + p->off_in[c & 1];
        wait(si, 2 + (c & 1));
        (void)hipMemcpyAsync(buf, static_cast<const char*>(o.h_data) + (size_t)t0 * proj * db,
                             (size_t)nt * proj * db, hipMemcpyHostToDevice, si);
        rec(c & 1, si);
        wait(s, c & 1);
        absmax_partial(kp, buf, (size_t)nt * proj, p->opts.data_dtype, ABSMAX_BLOCKS, c > 0, s);
        rec(2 + (c & 1), s);
      }
      hipLaunchKernelGGL(k_absmax_final, dim3(1), dim3(256), 0, s, const_cast<float*>(kp.dyn),
                         ABSMAX_BLOCKS, 0.f);
    }
  }
  float2* phase = nullptr;
  if (o.center_shift != 0.0) {
    phase = reinterpret_cast<float2*>(work + p->off_phase);
    hipLaunchKernelGGL(k_axis_phase, dim3(cdiv(p->w_p, 256)), dim3(256), 0, s, phase, p->w_p,
                       o.center_shift);
  }
  float2* W1 = reinterpret_cast<float2*>(work + p->off_w1);
  void* D = work + p->off_D;
  float2* G = reinterpret_cast<float2*>(work + p->off_G);
  void* g = work + p->off_g;
  char* hD = hsp + p->off_hD;
  char* hg = hsp + p->off_hg;

  // ---- detector stage: per projection chunk
  const int cp = std::min(fft_capacity(p->h_p) / p->h_p, std::max(1, (p->w + 1) / 2));
  const int rows_w = std::min(fft_capacity(p->w_p) / p->w_p, p->n_slab);
  const size_t lds_h = (size_t)fft_capacity(p->h_p) * sizeof(float2);
  const size_t lds_w = (size_t)fft_capacity(p->w_p) * sizeof(float2);
  const size_t lds_g = (size_t)fft_capacity(p->grid) * sizeof(float2);
  const size_t lds_gc = (size_t)col_capacity(p->grid) * sizeof(float2);
  for (int t0 = 0, c = 0; t0 < p->n_theta; t0 += p->theta_chunk, ++c) {
    const int nt = std::min(p->theta_chunk, p->n_theta - t0);
    const void* src = d_data;
    int src_th0 = 0;
    if (host_in) {
      char* buf = io + p->off_in[c & 1];
      wait(si, 2 + (c & 1));
      (void)hipMemcpyAsync(buf, static_cast<const char*>(o.h_data) + (size_t)t0 * proj * db,
                           (size_t)nt * proj * db, hipMemcpyHostToDevice, si);
      rec(c & 1, si);
      wait(s, c & 1);
      src = buf;
      src_th0 = t0;
    }
    void* Dt = D;
    int d_nth = p->n_theta, d_th0 = 0;
    if (p->spill_D) {
      Dt = work + p->off_Dout[c & 1];
      d_nth = p->theta_chunk;
      d_th0 = t0;
      wait(s, 6 + (c & 1));
    }
    {
      StageTimer timer(p, s, LAMINO_STAGE_DETECTOR, 2, timing);
      if (p->h_p == 512)
        hipLaunchKernelGGL((k_proj_cols_fwd_w<8, WFFT_CW_DET>), dim3(cdiv(p->w, 2 * WFFT_CW_DET), nt), dim3(512), 0, s, kp,
                           src, W1, t0, src_th0);
      else if (p->h_p == 1024)
        hipLaunchKernelGGL((k_proj_cols_fwd_w<16, WFFT_CW_DET>), dim3(cdiv(p->w, 2 * WFFT_CW_DET), nt), dim3(512), 0, s, kp,
                           src, W1, t0, src_th0);
      else
        hipLaunchKernelGGL(FFT_KERNEL(k_proj_cols_fwd, p->h_p), dim3(cdiv(p->w, 2 * cp), nt), dim3(NTF), lds_h, s, kp, src,
                           W1, t0, cp, src_th0);
      if (host_in) rec(2 + (c & 1), s);
      if (p->w_p == 512)
        hipLaunchKernelGGL(k_proj_rows_fwd_w<8>, dim3(cdiv(p->n_slab, WFFT_WAVES * WFFT_ROWS), nt),
                           dim3(64 * WFFT_WAVES), 0, s, kp, (const float2*)W1, Dt, kp.filt,
                           (const float2*)phase, t0, WFFT_ROWS, d_nth, d_th0);
      else if (p->w_p == 1024)
        hipLaunchKernelGGL(k_proj_rows_fwd_w<16>, dim3(cdiv(p->n_slab, WFFT_WAVES * WFFT_ROWS), nt),
                           dim3(64 * WFFT_WAVES), 0, s, kp, (const float2*)W1, Dt, kp.filt,
                           (const float2*)phase, t0, WFFT_ROWS, d_nth, d_th0);
      else
        hipLaunchKernelGGL(FFT_KERNEL(k_proj_rows_fwd, p->w_p), dim3(cdiv(p->n_slab, rows_w), nt), dim3(NTF), lds_w, s, kp,
                           (const float2*)W1, Dt, kp.filt, (const float2*)phase, t0, rows_w, d_nth,
                           d_th0);
    }
    if (p->spill_D) {
      // D[l][t0 .. t0 + nt)[k] of every slab l into the host spectra
      rec(4 + (c & 1), s);
      wait(so, 4 + (c & 1));
      const size_t wrow = (size_t)p->w_p * sb;
      (void)hipMemcpy2DAsync(hD + (size_t)t0 * wrow, (size_t)p->n_theta * wrow, Dt,
                             (size_t)p->theta_chunk * wrow, (size_t)nt * wrow, p->n_slab,
                             hipMemcpyDeviceToHost, so);
      rec(6 + (c & 1), so);
    }
  }
  if (p->spill_D) {
    // the host spectra are complete before any slab chunk is read back
    rec(9, so);
    wait(si, 9);
  }

  // ---- gridding and slab stages: per slab chunk
  const int rows_g = std::min(fft_capacity(p->grid) / p->grid, p->grid);
  const int cols_g = std::min(col_capacity(p->grid) / p->grid, p->n);
  for (int s0 = 0, j = 0; s0 < p->n_slab; s0 += p->slab_chunk, ++j) {
    const int ns = std::min(p->slab_chunk, p->n_slab - s0);
    const void* Dg = D;
    int d_l0 = 0;
    if (p->spill_D) {
      char* buf = work + p->off_Din[j & 1];
      const size_t slab = (size_t)p->n_theta * p->w_p * sb;
      wait(si, 2 + (j & 1));
      (void)hipMemcpyAsync(buf, hD + (size_t)s0 * slab, (size_t)ns * slab, hipMemcpyHostToDevice, si);
      rec(j & 1, si);
      wait(s, j & 1);
      Dg = buf;
      d_l0 = s0;
    }
    {
      StageTimer timer(p, s, LAMINO_STAGE_GRIDDING, 1, timing);
      spread_dispatch(kp, Dg, G, s0, ns, d_l0, s);
    }
    if (p->spill_D) rec(2 + (j & 1), s);
    void* gt = g;
    int g_l0 = 0;
    if (p->spill_g) {
      gt = work + p->off_gout[j & 1];
      g_l0 = s0;
      wait(s, 6 + (j & 1));
    }
    {
      StageTimer timer(p, s, LAMINO_STAGE_SLAB, 2, timing);
      if (p->grid == 512)
        hipLaunchKernelGGL(k_grid_rows_inv_w<8>, dim3(512 / (WFFT_WAVES * WFFT_ROWS), ns), dim3(64 * WFFT_WAVES), 0, s,
                           kp, G, WFFT_ROWS);
      else if (p->grid == 1024)
        hipLaunchKernelGGL(k_grid_rows_inv_w<16>, dim3(1024 / (WFFT_WAVES * WFFT_ROWS), ns), dim3(64 * WFFT_WAVES), 0, s,
                           kp, G, WFFT_ROWS);
      else
        hipLaunchKernelGGL(FFT_KERNEL(k_grid_rows_inv, p->grid), dim3(cdiv(p->grid, rows_g), ns), dim3(NTF), lds_g, s, kp, G,
                           rows_g);
      if (p->grid == 512)
        hipLaunchKernelGGL((k_grid_cols_adj_w<8, WFFT_CW_SLAB>), dim3(cdiv(p->n, WFFT_CW_SLAB), ns), dim3(512), 0, s, kp,
                           (const float2*)G, gt, s0, g_l0);
      else if (p->grid == 1024)
        hipLaunchKernelGGL((k_grid_cols_adj_w<16, WFFT_CW_WIDE>), dim3(cdiv(p->n, WFFT_CW_WIDE), ns), dim3(512), 0, s, kp,
                           (const float2*)G, gt, s0, g_l0);
      else
        hipLaunchKernelGGL(FFT_KERNEL(k_grid_cols_adj, p->grid), dim3(cdiv(p->n, cols_g), ns), dim3(NTF), lds_gc, s,
                           kp, (const float2*)G, gt, s0, cols_g, g_l0);
    }
    if (p->spill_g) {
      rec(4 + (j & 1), s);
      wait(so, 4 + (j & 1));
      (void)hipMemcpyAsync(hg + (size_t)s0 * ncol * sb, gt, (size_t)ns * ncol * sb,
                           hipMemcpyDeviceToHost, so);
      rec(6 + (j & 1), so);
    }
  }

  // ---- x3 transform
  const int zb = o.z_first, ze = o.z_count < 0 ? p->nz : o.z_first + o.z_count;
  if (!p->spill_g) {
    // z chunks (host output: io_z slices per chunk through the staging buffer)
    const int zc = host_out ? p->io_z : p->z_chunk;
    for (int z0 = zb, k = 0; z0 < ze; z0 += zc, ++k) {
      const int nzc = std::min(zc, ze - z0);
      float* out = d_vol;
      int out_z0 = zb;
      if (host_out) {
        out = reinterpret_cast<float*>(io + p->off_vout[k & 1]);
        out_z0 = z0;
        wait(s, 6 + (k & 1));
      }
      {
        StageTimer timer(p, s, LAMINO_STAGE_X3, 1, timing);
        launch_x3_adj(kp, g, (int)ncol, out, (int)ncol, 0, (int)ncol, z0, nzc, out_z0, s);
      }
      if (host_out) {
        rec(4 + (k & 1), s);
        wait(so, 4 + (k & 1));
        (void)hipMemcpyAsync(o.h_vol + (size_t)(z0 - zb) * ncol, out, (size_t)nzc * ncol * 4,
                             hipMemcpyDeviceToHost, so);
        rec(6 + (k & 1), so);
      }
    }
  } else {
    // column chunks of all slices; the host slab planes are complete first
    rec(9, so);
    wait(si, 9);
    const int cc = p->col_chunk;
    const int nzo = ze - zb;
    for (int c0 = 0, k = 0; c0 < (int)ncol; c0 += cc, ++k) {
      const int ncc = std::min(cc, (int)ncol - c0);
      char* buf = work + p->off_gcol[k & 1];
      wait(si, 2 + (k & 1));
      (void)hipMemcpy2DAsync(buf, (size_t)cc * sb, hg + (size_t)c0 * sb, ncol * sb, (size_t)ncc * sb,
                             p->n_slab, hipMemcpyHostToDevice, si);
      rec(k & 1, si);
      wait(s, k & 1);
      float* out = d_vol;
      int v_ld = (int)ncol, vcol0 = c0;
      if (host_out) {
        out = reinterpret_cast<float*>(io + p->off_vout[k & 1]);
        v_ld = cc;
        vcol0 = 0;
        wait(s, 6 + (k & 1));
      }
      {
        StageTimer timer(p, s, LAMINO_STAGE_X3, 1, timing);
        launch_x3_adj(kp, buf, cc, out, v_ld, vcol0, ncc, zb, nzo, zb, s);
      }
      rec(2 + (k & 1), s);
      if (host_out) {
        rec(4 + (k & 1), s);
        wait(so, 4 + (k & 1));
        (void)hipMemcpy2DAsync(o.h_vol + c0, ncol * 4, out, (size_t)cc * 4, (size_t)ncc * 4, nzo,
                               hipMemcpyDeviceToHost, so);
        rec(6 + (k & 1), so);
      }
    }
  }
  if (piped) {
    // the call is complete on s once both copy streams have drained
    rec(8, si);
    rec(9, so);
    wait(s, 8);
    wait(s, 9);
  }
  return hipGetLastError();
}

hipError_t run_forward(const lamino_plan_s* p, const float* d_vol, void* d_data, hipStream_t s) {
  const KParams kp = make_params(p, false);
  float2* W1 = reinterpret_cast<float2*>(wptr(p, p->off_w1));
  void* D = wptr(p, p->off_D);
  float2* G = reinterpret_cast<float2*>(wptr(p, p->off_G));
  void* g = wptr(p, p->off_g);
  const int ncol = p->n * p->n;
  if (kp.dyn) input_factor(kp, d_vol, (size_t)p->nz * ncol, LAMINO_F32, 0.f, s);
  {
    StageTimer timer(p, s, LAMINO_STAGE_X3, 1);
    hipLaunchKernelGGL(k_x3_fwd_b, dim3(cdiv(ncol, 32 * X3B_WAVES), cdiv(2 * p->n_slab, X3B_ROWS)),
                       dim3(64 * X3B_WAVES), 0, s, kp, d_vol, g);
  }
  const int rows_g = std::min(fft_capacity(p->grid) / p->grid, p->grid);
  const int cols_g = std::min(col_capacity(p->grid) / p->grid, p->n);
  const size_t lds_h = (size_t)fft_capacity(p->h_p) * sizeof(float2);
  const size_t lds_w = (size_t)fft_capacity(p->w_p) * sizeof(float2);
  const size_t lds_g = (size_t)fft_capacity(p->grid) * sizeof(float2);
  const size_t lds_gc = (size_t)col_capacity(p->grid) * sizeof(float2);
  for (int s0 = 0; s0 < p->n_slab; s0 += p->slab_chunk) {
    const int ns = std::min(p->slab_chunk, p->n_slab - s0);
    {
      StageTimer timer(p, s, LAMINO_STAGE_SLAB, 2);
      if (p->grid == 512) {
        hipLaunchKernelGGL((k_grid_cols_fwd_w<8, WFFT_CW_SLAB>), dim3(cdiv(p->n, WFFT_CW_SLAB), ns), dim3(512), 0, s, kp,
                           (const void*)g, G, s0);
        hipLaunchKernelGGL(k_grid_rows_fwd_w<8>, dim3(512 / (WFFT_WAVES * WFFT_ROWS), ns), dim3(64 * WFFT_WAVES), 0, s,
                           kp, G, WFFT_ROWS);
      } else if (p->grid == 1024) {
        hipLaunchKernelGGL((k_grid_cols_fwd_w<16, WFFT_CW_WIDE>), dim3(cdiv(p->n, WFFT_CW_WIDE), ns), dim3(512), 0, s, kp,
                           (const void*)g, G, s0);
        hipLaunchKernelGGL(k_grid_rows_fwd_w<16>, dim3(1024 / (WFFT_WAVES * WFFT_ROWS), ns), dim3(64 * WFFT_WAVES), 0, s,
                           kp, G, WFFT_ROWS);
      } else {
        hipLaunchKernelGGL(FFT_KERNEL(k_grid_cols_fwd, p->grid), dim3(cdiv(p->n, cols_g), ns), dim3(NTF), lds_gc, s, kp,
                           (const void*)g, G, s0, cols_g);
        hipLaunchKernelGGL(FFT_KERNEL(k_grid_rows_fwd, p->grid), dim3(cdiv(p->grid, rows_g), ns), dim3(NTF), lds_g, s, kp,
                           G, rows_g);
      }
    }
    StageTimer timer(p, s, LAMINO_STAGE_GRIDDING, 1);
    interp_dispatch(kp, G, D, s0, ns, s);
  }
  const int cp = std::min(fft_capacity(p->h_p) / p->h_p, std::max(1, (p->w + 1) / 2));
  const int rows_w = std::min(fft_capacity(p->w_p) / p->w_p, p->n_slab);
  // 1 / (h_p w_p) of the inverse DFT, and the static float16 factors removed
  const float scale = (float)(1.0 / ((double)p->h_p * p->w_p) / ((double)kp.fwd_g_scale * kp.fwd_D_scale));
  for (int t0 = 0; t0 < p->n_theta; t0 += p->theta_chunk) {
    const int nt = std::min(p->theta_chunk, p->n_theta - t0);
    StageTimer timer(p, s, LAMINO_STAGE_DETECTOR, 2);
    if (p->w_p == 512)
      hipLaunchKernelGGL(k_proj_rows_inv_w<8>, dim3(cdiv(p->n_slab, WFFT_WAVES * WFFT_ROWS), nt), dim3(64 * WFFT_WAVES),
                         0, s, kp, (const void*)D, W1, t0, WFFT_ROWS);
    else if (p->w_p == 1024)
      hipLaunchKernelGGL(k_proj_rows_inv_w<16>, dim3(cdiv(p->n_slab, WFFT_WAVES * WFFT_ROWS), nt), dim3(64 * WFFT_WAVES),
                         0, s, kp, (const void*)D, W1, t0, WFFT_ROWS);
    else
      hipLaunchKernelGGL(FFT_KERNEL(k_proj_rows_inv, p->w_p), dim3(cdiv(p->n_slab, rows_w), nt), dim3(NTF), lds_w, s, kp,
                         (const void*)D, W1, t0, rows_w);
    if (p->h_p == 512)
      hipLaunchKernelGGL((k_proj_cols_inv_w<8, WFFT_CW_DET>), dim3(cdiv(p->w, 2 * WFFT_CW_DET), nt), dim3(512), 0, s, kp,
                         (const float2*)W1, d_data, t0, scale);
    else if (p->h_p == 1024)
      hipLaunchKernelGGL((k_proj_cols_inv_w<16, WFFT_CW_DET>), dim3(cdiv(p->w, 2 * WFFT_CW_DET), nt), dim3(512), 0, s, kp,
                         (const float2*)W1, d_data, t0, scale);
    else
      hipLaunchKernelGGL(FFT_KERNEL(k_proj_cols_inv, p->h_p), dim3(cdiv(p->w, 2 * cp), nt), dim3(NTF), lds_h, s, kp,
                         (const float2*)W1, d_data, t0, cp, scale);
  }
  return hipGetLastError();
}

}  // namespace lam
