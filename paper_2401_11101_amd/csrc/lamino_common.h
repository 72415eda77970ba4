// Shared host/device helpers of the laminography library.
//
// Everything here is plain arithmetic on indices and float2 values, usable
// from the gfx950 kernels and from host unit tests of the index logic.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#define LAM_HD __host__ __device__ __forceinline__

namespace lam {

// ---------------------------------------------------------------- complex
LAM_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
LAM_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
LAM_HD float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
LAM_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
LAM_HD float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
LAM_HD float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }
LAM_HD float2 mul_pi(float2 a) { return make_float2(-a.y, a.x); }

// e / d for 0 <= e < 2^24 and 1 <= d < 2^24, given inv = 1.0f / d: the
// float product is within one of the quotient, and one correction step
// makes it exact.  A handful of instructions instead of the generic 32-bit
// integer division (checked exhaustively over small ranges by the host
// self-test).
LAM_HD int div24(int e, int d, float inv) {
  int q = (int)((float)e * inv);
  const int r = e - q * d;
  q += (r >= d) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

LAM_HD int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// ------------------------------------------------------------ FFT passes
// Stockham autosort FFT of length N = 2^log2N: radix-8 passes, then one
// radix-4 or radix-2 pass for the remaining bits.  A pass with sub-transform
// size Ns maps butterfly j (0 <= j < N/R) from positions j + r N/R to
// positions (j - j%Ns) R + j%Ns + q Ns after twiddling input r by
// w^(r (j%Ns)), w = exp(-+2 pi i / (Ns R)).  The twiddle table holds
// tw[t] = exp(-2 pi i t / Nmax), Nmax = 2^log2max >= N.

struct FftPass {
  int radix;   // 8, 4 or 2
  int log2Ns;  // log2 of the sub-transform size before this pass
};

constexpr LAM_HD int fft_num_passes(int log2N) { return log2N / 3 + (log2N % 3 ? 1 : 0); }

constexpr LAM_HD FftPass fft_pass(int log2N, int p) {
  FftPass f{};
  const int n8 = log2N / 3;
  if (p < n8) {
    f.radix = 8;
    f.log2Ns = 3 * p;
  } else {
    f.radix = (log2N % 3 == 2) ? 4 : 2;
    f.log2Ns = 3 * n8;
  }
  return f;
}

LAM_HD float2 twiddle(const float2* tw, int idx, bool inv) {
  float2 t = tw[idx];
  return inv ? cconj(t) : t;
}

// Inputs of butterfly j of a radix-4 pass over one transform at `a`.
LAM_HD void r4_load(const float2* a, int N, int j, float2 v[4]) {
  const int q = N >> 2;
  v[0] = a[j];
  v[1] = a[j + q];
  v[2] = a[j + 2 * q];
  v[3] = a[j + 3 * q];
}

// Twiddle and 4-point DFT of butterfly j in registers; outputs in v[q].
LAM_HD void r4_compute(int j, int log2Ns, const float2* tw, int log2max, bool inv, float2 v[4]) {
  const int Ns = 1 << log2Ns;
  const int k = j & (Ns - 1);
  if (Ns > 1) {
    const int sh = log2max - (log2Ns + 2);
    v[1] = cmul(v[1], twiddle(tw, k << sh, inv));
    v[2] = cmul(v[2], twiddle(tw, (2 * k) << sh, inv));
    v[3] = cmul(v[3], twiddle(tw, (3 * k) << sh, inv));
  }
  const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  const float2 s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
  const float2 rot = inv ? mul_pi(d13) : mul_mi(d13);
  v[0] = cadd(s02, s13);
  v[1] = cadd(d02, rot);
  v[2] = csub(s02, s13);
  v[3] = csub(d02, rot);
}

// Output q of butterfly j goes to (j - j%Ns) R + j%Ns + q Ns.
template <int R>
LAM_HD void rstore(float2* a, int j, int log2Ns, const float2* v) {
  const int Ns = 1 << log2Ns;
  const int k = j & (Ns - 1);
  const int o = (j - k) * R + k;
  for (int q = 0; q < R; ++q) a[o + q * Ns] = v[q];
}

LAM_HD void r4_compute_store(float2* a, int j, int log2Ns, const float2* tw, int log2max,
                             bool inv, float2 v[4]) {
  r4_compute(j, log2Ns, tw, log2max, inv, v);
  rstore<4>(a, j, log2Ns, v);
}

LAM_HD void r8_load(const float2* a, int N, int j, float2 v[8]) {
  const int q = N >> 3;
  for (int r = 0; r < 8; ++r) v[r] = a[j + r * q];
}

// 4-point DFT in place (forward: exp(-2 pi i rq/4); inverse: conjugate).
LAM_HD void dft4(float2& x0, float2& x1, float2& x2, float2& x3, bool inv) {
  const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2);
  const float2 s13 = cadd(x1, x3), d13 = csub(x1, x3);
  const float2 rot = inv ? mul_pi(d13) : mul_mi(d13);
  x0 = cadd(s02, s13);
  x2 = csub(s02, s13);
  x1 = cadd(d02, rot);
  x3 = csub(d02, rot);
}

LAM_HD void r8_compute(int j, int log2Ns, const float2* tw, int log2max, bool inv, float2 v[8]) {
  const int Ns = 1 << log2Ns;
  const int k = j & (Ns - 1);
  if (Ns > 1) {
    const int sh = log2max - (log2Ns + 3);
    for (int r = 1; r < 8; ++r) v[r] = cmul(v[r], twiddle(tw, (r * k) << sh, inv));
  }
  // 8-point DFT: 4-point DFTs of the even and odd inputs, then combine with
  // w8^q, w8 = exp(-+2 pi i / 8)
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3, inv);
  dft4(o0, o1, o2, o3, inv);
  const float h = 0.70710678118654752f;
  // o1 *= w8, o2 *= w8^2, o3 *= w8^3
  o1 = inv ? make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y))
           : make_float2(h * (o1.x + o1.y), h * (o1.y - o1.x));
  o2 = inv ? mul_pi(o2) : mul_mi(o2);
  o3 = inv ? make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y))
           : make_float2(h * (o3.y - o3.x), -h * (o3.x + o3.y));
  v[0] = cadd(e0, o0);
  v[1] = cadd(e1, o1);
  v[2] = cadd(e2, o2);
  v[3] = cadd(e3, o3);
  v[4] = csub(e0, o0);
  v[5] = csub(e1, o1);
  v[6] = csub(e2, o2);
  v[7] = csub(e3, o3);
}

LAM_HD void r8_compute_store(float2* a, int j, int log2Ns, const float2* tw, int log2max,
                             bool inv, float2 v[8]) {
  r8_compute(j, log2Ns, tw, log2max, inv, v);
  rstore<8>(a, j, log2Ns, v);
}

LAM_HD void r2_load(const float2* a, int N, int j, float2 v[2]) {
  v[0] = a[j];
  v[1] = a[j + (N >> 1)];
}

LAM_HD void r2_compute(int j, int log2Ns, const float2* tw, int log2max, bool inv, float2 v[2]) {
  const int Ns = 1 << log2Ns;
  const int k = j & (Ns - 1);
  if (Ns > 1) v[1] = cmul(v[1], twiddle(tw, k << (log2max - (log2Ns + 1)), inv));
  const float2 s = cadd(v[0], v[1]), d = csub(v[0], v[1]);
  v[0] = s;
  v[1] = d;
}

LAM_HD void r2_compute_store(float2* a, int j, int log2Ns, const float2* tw, int log2max,
                             bool inv, float2 v[2]) {
  r2_compute(j, log2Ns, tw, log2max, inv, v);
  rstore<2>(a, j, log2Ns, v);
}

// ---------------------------------------------------- sample positions
// Slab l of the tilted grid (eq:uneqspace): the sample of angle theta and
// detector frequency m sits at (X, Y) = N_g (xi1, xi2) grid cells with
//   X = (N_g / w_p) cos(t) m + (N_g l sin(p) / h_p) sin(t)
//   Y = (N_g / w_p) sin(t) m - (N_g l sin(p) / h_p) cos(t).
// Every kernel computes it with this function so that gridding and
// interpolation see bit-identical positions.
LAM_HD void sample_pos(float ncw, float gcl, float2 cs, int m, float& X, float& Y) {
  const float fm = (float)m;
  X = fmaf(ncw * cs.x, fm, gcl * cs.y);
  Y = fmaf(ncw * cs.y, fm, -(gcl * cs.x));
}

// m-interval of samples whose coordinate a m + b lies in [lo, hi), as
// sample_pos computes it (one fma); returns false if empty.  Conservative:
// the bounds t0, t1 carry three roundings (relative 2^-24 each), and a
// sample's computed coordinate is off by at most 2^-24 of its magnitude,
// i.e. by that over |a| in m.  floor / ceil absorb a total error below one
// sample; the margin mg adds whole samples beyond that (4x the bound), and
// is 0 unless |a| is tiny.
LAM_HD bool coord_interval(float a, float b, float lo, float hi, int& mlo, int& mhi) {
  if (fabsf(a) < 1e-6f) {
    if (b >= lo - 1.0f && b < hi + 1.0f) {
      mlo = -(1 << 30);
      mhi = 1 << 30;
      return true;
    }
    return false;
  }
  const float ia = 1.0f / a;
  float t0 = (lo - b) * ia, t1 = (hi - b) * ia;
  if (t0 > t1) {
    const float t = t0;
    t0 = t1;
    t1 = t;
  }
  // clamp before the conversion so that nothing overflows an int
  t0 = fmaxf(t0, -1.0e8f);
  t1 = fminf(t1, 1.0e8f);
  const float xmax = fmaxf(fabsf(lo), fabsf(hi)) + 1.0f;
  const float err = 4.0f * (6.0e-8f * xmax * fabsf(ia) + 1.8e-7f * fmaxf(fabsf(t0), fabsf(t1)));
  const int mg = (int)fminf(err, 1.0e6f);
  mlo = (int)floorf(t0) - mg;
  mhi = (int)ceilf(t1) + mg;
  return mlo <= mhi;
}

// Candidate samples of one angle for a tile copy [x0, x0 + ext) x
// [y0, y0 + ext): returns the m-range [mlo, mhi] (inclusive) within the
// stored frequencies -(w_p/2 - 1) .. w_p/2 - 1.
LAM_HD bool tile_candidates(float ncw, float gcl, float2 cs, float x0, float y0, float extx,
                            float exty, int half_m, int& mlo, int& mhi) {
  int a0, a1, b0, b1;
  if (!coord_interval(ncw * cs.x, gcl * cs.y, x0, x0 + extx, a0, a1)) return false;
  if (!coord_interval(ncw * cs.y, -(gcl * cs.x), y0, y0 + exty, b0, b1)) return false;
  mlo = a0 > b0 ? a0 : b0;
  mhi = a1 < b1 ? a1 : b1;
  if (mlo < -half_m) mlo = -half_m;
  if (mhi > half_m) mhi = half_m;
  return mlo <= mhi;
}

// Tile order for the gridding launches: rank 0 .. ntx^2 - 1 -> tile (tx, ty)
// in square rings around the grid centre, innermost first.  Samples are
// densest near the centre (polar sampling), so the longest-running tiles
// start first.  ntx is 1 or even.
LAM_HD void ring_tile(int rank, int ntx, int& tx, int& ty) {
  if (ntx == 1) {
    tx = ty = 0;
    return;
  }
  int k = 0;  // ring k holds ranks (2k)^2 .. (2k + 2)^2 - 1
  while ((2 * k + 2) * (2 * k + 2) <= rank) ++k;
  const int q = rank - 4 * k * k;
  const int s = 2 * k + 2;  // side of the ring
  const int lo = ntx / 2 - 1 - k, hi = ntx / 2 + k;
  if (q < s) {
    tx = lo + q;
    ty = lo;
  } else if (q < 2 * s - 1) {
    tx = hi;
    ty = lo + 1 + (q - s);
  } else if (q < 3 * s - 2) {
    tx = hi - 1 - (q - (2 * s - 1));
    ty = hi;
  } else {
    tx = lo;
    ty = hi - 1 - (q - (3 * s - 2));
  }
}

// Tile of a volume stencil kernel launched on `grid` blocks (a multiple of
// 8): hardware block b runs on XCD b % 8, so block b takes tile
// (b % 8) * (grid / 8) + b / 8 and each XCD walks one contiguous run of the
// nb tiles (x tiles fastest, then y, then z).  Returns false for the
// padding blocks past nb.
LAM_HD bool xcd_tile(int b, int grid, int nb, int nbx, int nby, int& bx, int& by, int& bz) {
  const int t = (b & 7) * (grid >> 3) + (b >> 3);
  if (t >= nb) return false;
  bx = t % nbx;
  const int r = t / nbx;
  by = r % nby;
  bz = r / nby;
  return true;
}

// Wrap an integer grid coordinate to [-N/2, N/2) (N a power of two).
LAM_HD int wrap_centred(int k, int N) { return ((k + (N >> 1)) & (N - 1)) - (N >> 1); }

}  // namespace lam
