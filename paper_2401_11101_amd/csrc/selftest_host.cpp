// Host-only checks of the index logic the kernels share (no GPU needed).
//
//  fft     Stockham radix-8/4/2 passes of lamino_common.h, run serially over
//          ping-pong buffers, against a naive double-precision DFT for
//          N = 2 .. 8192, both directions.
//  cand    for random slabs, angles and tiles: every sample whose Gaussian
//          taps reach a tile copy lies in that copy's candidate m-interval
//          (gridding), and every sample is owned by exactly one tile through
//          its wrapped base cell, inside that tile's candidate interval
//          (interpolation).
//  ring    the centre-out tile order is a bijection onto the ntx x ntx tiles.
//  div24   the float-reciprocal integer division equals e / d.
//  xcd     the XCD-grouped tile order of the volume stencil kernels (64 x 4
//          x 16 voxel tiles) covers every voxel of ragged volumes exactly
//          once, and each XCD's tiles form one contiguous run.
// Prints one line per check and exits non-zero on the first failure.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "lamino_common.h"

using namespace lam;

static int check_fft() {
  const int log2max = 13;
  const int Nmax = 1 << log2max;
  std::vector<float2> tw(Nmax);
  for (int t = 0; t < Nmax; ++t) {
    const double a = -2.0 * M_PI * t / Nmax;
    tw[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::mt19937 rng(1);
  std::normal_distribution<float> nd;
  for (int log2N = 1; log2N <= log2max; ++log2N) {
    const int N = 1 << log2N;
    for (int inv = 0; inv < 2; ++inv) {
      std::vector<float2> a(N), b(N), x(N);
      for (int i = 0; i < N; ++i) x[i] = a[i] = make_float2(nd(rng), nd(rng));
      float2* src = a.data();
      float2* dst = b.data();
      for (int p = 0; p < fft_num_passes(log2N); ++p) {
        const FftPass f = fft_pass(log2N, p);
        for (int j = 0; j < N / f.radix; ++j) {
          if (f.radix == 8) {
            float2 v[8];
            r8_load(src, N, j, v);
            r8_compute_store(dst, j, f.log2Ns, tw.data(), log2max, inv, v);
          } else if (f.radix == 4) {
            float2 v[4];
            r4_load(src, N, j, v);
            r4_compute_store(dst, j, f.log2Ns, tw.data(), log2max, inv, v);
          } else {
            float2 v[2];
            r2_load(src, N, j, v);
            r2_compute_store(dst, j, f.log2Ns, tw.data(), log2max, inv, v);
          }
        }
        std::swap(src, dst);
      }
      double err = 0, ref = 0;
      const double sgn = inv ? 1.0 : -1.0;
      const int stride = N > 512 ? N / 64 : 1;  // naive DFT on a subset of bins when large
      for (int k = 0; k < N; k += stride) {
        std::complex<double> s = 0;
        for (int n = 0; n < N; ++n)
          s += std::complex<double>(x[n].x, x[n].y) *
               std::polar(1.0, sgn * 2.0 * M_PI * (double)((long)k * n % N) / N);
        err += std::norm(s - std::complex<double>(src[k].x, src[k].y));
        ref += std::norm(s);
      }
      const double rel = std::sqrt(err / ref);
      if (!(rel < 2e-6)) {
        std::printf("fft N=%d inv=%d rel=%.3e FAIL\n", N, inv, rel);
        return 1;
      }
    }
  }
  std::printf("fft ok\n");
  return 0;
}

static int check_candidates() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> U(0, 1);
  const int cases[][4] = {{16, 16, 32, 3}, {64, 128, 64, 5}, {128, 256, 128, 2},
                          {512, 512, 512, 6}, {256, 256, 128, 8}, {32, 64, 16, 4}};
  for (auto& c : cases) {
    const int grid = c[0], wp = c[1], hp = c[2], M = c[3];
    const int tile = grid <= 128 ? (grid < 32 ? grid : 32) : 64;
    const int ntx = grid / tile;
    for (int rep = 0; rep < 3; ++rep) {
      const double phi = (U(rng) * 2 - 1) * 1.3;
      const float ncw = (float)((double)grid / wp);
      const float gs = (float)((double)grid * std::sin(phi) / hp);
      const int half_m = wp / 2 - 1;
      for (int it = 0; it < 40; ++it) {
        const int l = (int)(U(rng) * (hp / 2));
        // the first angles lie next to pi/2 (tiny |cos|: the widest margins)
        static const double near[8] = {0.0, 1e-7, -3e-6, 8e-6, -2e-5, 1e-4, -7e-4, 3e-3};
        const double th = it < 8 ? M_PI / 2 + near[it] : U(rng) * 2 * M_PI;
        const float2 cs = make_float2((float)std::cos(th), (float)std::sin(th));
        const float gcl = gs * (float)l;
        std::vector<int> owners(2 * half_m + 1, 0);
        for (int t = 0; t < ntx * ntx; ++t) {
          const int X0 = -grid / 2 + (t % ntx) * tile, Y0 = -grid / 2 + (t / ntx) * tile;
          for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx) {
              int mlo = 1, mhi = 0, olo = 1, ohi = 0;
              tile_candidates(ncw, gcl, cs, (float)(X0 + sx * grid) - M, (float)(Y0 + sy * grid) - M,
                              (float)(tile + 2 * M - 1), (float)(tile + 2 * M - 1), half_m, mlo, mhi);
              tile_candidates(ncw, gcl, cs, (float)(X0 + sx * grid), (float)(Y0 + sy * grid),
                              (float)tile, (float)tile, half_m, olo, ohi);
              for (int m = -half_m; m <= half_m; ++m) {
                float X, Y;
                sample_pos(ncw, gcl, cs, m, X, Y);
                const int bx = (int)std::floor(X) - M + 1 - sx * grid - X0;
                const int by = (int)std::floor(Y) - M + 1 - sy * grid - Y0;
                const bool reach = !(bx + 2 * M <= 0 || bx >= tile || by + 2 * M <= 0 || by >= tile);
                if (reach && (m < mlo || m > mhi)) {
                  std::printf("cand spread miss grid=%d M=%d l=%d th=%f m=%d FAIL\n", grid, M, l, th, m);
                  return 1;
                }
                const int wx = wrap_centred((int)std::floor(X), grid) - X0;
                const int wy = wrap_centred((int)std::floor(Y), grid) - Y0;
                const bool own = wx >= 0 && wx < tile && wy >= 0 && wy < tile;
                const bool here = (int)std::floor(X) - sx * grid - X0 == wx &&
                                  (int)std::floor(Y) - sy * grid - Y0 == wy;
                if (own && here) {
                  if (m < olo || m > ohi) {
                    std::printf("cand interp miss grid=%d l=%d m=%d FAIL\n", grid, l, m);
                    return 1;
                  }
                  owners[m + half_m]++;
                }
              }
            }
        }
        for (int m = -half_m; m <= half_m; ++m)
          if (owners[m + half_m] != 1) {
            std::printf("cand ownership grid=%d m=%d owners=%d FAIL\n", grid, m, owners[m + half_m]);
            return 1;
          }
      }
    }
  }
  std::printf("cand ok\n");
  return 0;
}

static int check_ring_order() {
  for (int ntx = 1; ntx <= 128; ntx = ntx == 1 ? 2 : 2 * ntx) {
    std::vector<int> seen(ntx * ntx, 0);
    int prev = -1;
    for (int r = 0; r < ntx * ntx; ++r) {
      int tx, ty;
      ring_tile(r, ntx, tx, ty);
      if (tx < 0 || tx >= ntx || ty < 0 || ty >= ntx || seen[ty * ntx + tx]++) {
        std::printf("ring ntx=%d rank=%d -> (%d, %d) FAIL\n", ntx, r, tx, ty);
        return 1;
      }
      // Chebyshev distance from the centre never decreases along the order
      const int d = std::max(std::max(tx - ntx / 2, ntx / 2 - 1 - tx), std::max(ty - ntx / 2, ntx / 2 - 1 - ty));
      if (ntx > 1 && d < prev) {
        std::printf("ring ntx=%d rank=%d not centre-out FAIL\n", ntx, r);
        return 1;
      }
      prev = d;
    }
  }
  std::printf("ring ok\n");
  return 0;
}

static int check_div24() {
  // every numerator below 2^16 for every divisor up to 4200, then a sample
  // of numerators up to 2^24
  for (int d = 1; d <= 4200; ++d) {
    const float inv = 1.0f / (float)d;
    for (int e = 0; e < (1 << 16); ++e)
      if (div24(e, d, inv) != e / d) {
        std::printf("div24 %d / %d FAIL\n", e, d);
        return 1;
      }
  }
  std::mt19937 rng(7);
  for (int t = 0; t < 20000000; ++t) {
    const int d = 1 + (int)(rng() % ((1u << 24) - 1));
    const int e = (int)(rng() % (1u << 24));
    if (div24(e, d, 1.0f / (float)d) != e / d) {
      std::printf("div24 %d / %d FAIL\n", e, d);
      return 1;
    }
  }
  std::printf("div24 ok\n");
  return 0;
}

static int check_xcd_tiles() {
  const int shapes[][3] = {{1, 1, 1}, {16, 4, 64}, {7, 9, 130}, {33, 65, 65}, {256, 256, 256},
                           {17, 3, 200}, {512, 1024, 1024}};
  for (const auto& sh : shapes) {
    const int nz = sh[0], ny = sh[1], nx = sh[2];
    const int nbx = (nx + 63) / 64, nby = (ny + 3) / 4, nbz = (nz + 15) / 16;
    const int nb = nbx * nby * nbz, grid = 8 * ((nb + 7) / 8);
    std::vector<unsigned char> seen((size_t)nb, 0);
    std::vector<int> first(8, -1), last(8, -1);
    size_t voxels = 0;
    for (int b = 0; b < grid; ++b) {
      int bx, by, bz;
      if (!xcd_tile(b, grid, nb, nbx, nby, bx, by, bz)) continue;
      if (bx < 0 || bx >= nbx || by < 0 || by >= nby || bz < 0 || bz >= nbz) {
        std::printf("xcd %dx%dx%d block %d out of range FAIL\n", nz, ny, nx, b);
        return 1;
      }
      const int t = (bz * nby + by) * nbx + bx;
      if (seen[t]++) {
        std::printf("xcd %dx%dx%d tile %d twice FAIL\n", nz, ny, nx, t);
        return 1;
      }
      // each XCD's successive blocks take successive tiles
      const int x = b & 7;
      if (last[x] >= 0 && t != last[x] + 1) {
        std::printf("xcd %dx%dx%d XCD %d not contiguous FAIL\n", nz, ny, nx, x);
        return 1;
      }
      if (first[x] < 0) first[x] = t;
      last[x] = t;
      voxels += (size_t)std::min(64, nx - bx * 64) * std::min(4, ny - by * 4) *
                std::min(16, nz - bz * 16);
    }
    if (voxels != (size_t)nx * ny * nz) {
      std::printf("xcd %dx%dx%d covers %zu voxels FAIL\n", nz, ny, nx, voxels);
      return 1;
    }
  }
  std::printf("xcd ok\n");
  return 0;
}

int main() {
  if (check_fft()) return 1;
  if (check_candidates()) return 1;
  if (check_ring_order()) return 1;
  if (check_xcd_tiles()) return 1;
  if (check_div24()) return 1;
  return 0;
}
