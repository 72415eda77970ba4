// Total-variation regularised reconstruction (Appendix A): the finite
// difference operators, the isotropic soft threshold with the dual update,
// and an ADMM driver whose inner conjugate-gradient solve keeps every
// scalar on the device.
//
// Discretisation (the paper gives the continuous operators only):
//   grad mu = forward differences along x, y, z, the last difference
//             along each axis set to zero;          out[c][z][y][x], c = x, y, z
//   div p   = -grad^T p (backward differences with matching boundary terms).
// The psi-step is the minimiser of the augmented Lagrangian eq:alagr as
// written: psi = shrink(grad mu + lambda / rho, alpha / rho) per voxel on
// the 3-vector, then lambda += rho (grad mu - psi) (eq:lamd).
//
// Memory traffic.  Every kernel streams the volume once: a 256-thread block
// owns a 64 (x) by 4 (y) column of voxels over TV_ZB consecutive z planes,
// so the x, y and z neighbours of a stencil are re-read from L1/L2 rather
// than HBM.  Hardware block ids are dealt to the 8 XCDs round robin; the
// tile index is remapped so that each XCD walks one contiguous run of
// tiles and the halo planes of neighbouring tiles meet in the same L2.
//
// Reductions (the CG inner products) accumulate in double precision per
// thread, reduce per block into a partials array (one slot per block, zero
// for idle blocks) and are summed by a one-block finalize kernel in a fixed
// order, so results are deterministic.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lamino_common.h"
#include "lamino_internal.h"

namespace lam {
namespace {

constexpr int TV_BX = 64;   // voxels along x per block (one wavefront)
constexpr int TV_BY = 4;    // rows per block (one wavefront each)
constexpr int TV_ZB = 16;   // z planes per block
constexpr int TV_NT = TV_BX * TV_BY;
constexpr int TV_FIN = 256; // threads of the finalize kernel

struct Vol3 {
  int nx, ny, nz;
  int nbx, nby, nbz;
  int nb;        // tiles
  int grid;      // hardware blocks: 8 * ceil(nb / 8)
  size_t plane;  // nx * ny
  size_t nv;     // nx * ny * nz
};

Vol3 vol3(int nz, int ny, int nx) {
  Vol3 d;
  d.nx = nx;
  d.ny = ny;
  d.nz = nz;
  d.nbx = (nx + TV_BX - 1) / TV_BX;
  d.nby = (ny + TV_BY - 1) / TV_BY;
  d.nbz = (nz + TV_ZB - 1) / TV_ZB;
  d.nb = d.nbx * d.nby * d.nbz;
  d.grid = 8 * ((d.nb + 7) / 8);
  d.plane = (size_t)nx * ny;
  d.nv = d.plane * nz;
  return d;
}

// Voxel coordinates of this thread's column; false for the padding blocks
// that round the grid up to a multiple of the XCD count.
__device__ __forceinline__ bool tile_origin(const Vol3& d, int& x, int& y, int& z0) {
  int bx, by, bz;
  if (!xcd_tile(blockIdx.x, d.grid, d.nb, d.nbx, d.nby, bx, by, bz)) return false;
  x = bx * TV_BX + (threadIdx.x & (TV_BX - 1));
  y = by * TV_BY + (threadIdx.x / TV_BX);
  z0 = bz * TV_ZB;
  return true;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block sum of two values into partials[2 * blockIdx.x + {0, 1}].
__device__ __forceinline__ void block_sum2(double a, double b, double* partials) {
  __shared__ double red[2][TV_NT / 64];
  a = wave_sum(a);
  b = wave_sum(b);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wv] = a;
    red[1][wv] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < TV_NT / 64; ++i) {
      sa += red[0][i];
      sb += red[1][i];
    }
    partials[2 * blockIdx.x] = sa;
    partials[2 * blockIdx.x + 1] = sb;
  }
}

// ---------------------------------------------------------------------------
// Operators

__global__ __launch_bounds__(TV_NT) void k_tv_grad(const float* __restrict__ mu,
                                                    float* __restrict__ out, Vol3 d) {
  int x, y, z0;
  if (!tile_origin(d, x, y, z0) || x >= d.nx || y >= d.ny) return;
  const int z1 = min(z0 + TV_ZB, d.nz);
  const size_t ox = x + 1 < d.nx ? 1 : 0;
  const size_t oy = y + 1 < d.ny ? d.nx : 0;
  size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
  float c = mu[v];
  for (int z = z0; z < z1; ++z, v += d.plane) {
    const size_t oz = z + 1 < d.nz ? d.plane : 0;
    const float ax = mu[v + ox], ay = mu[v + oy], az = mu[v + oz];
    // a clamped neighbour equals the centre: the boundary difference is 0
    out[v] = ax - c;
    out[v + d.nv] = ay - c;
    out[v + 2 * d.nv] = az - c;
    c = az;
  }
}

__global__ __launch_bounds__(TV_NT) void k_tv_div(const float* __restrict__ p,
                                                   float* __restrict__ out, Vol3 d) {
  int x, y, z0;
  if (!tile_origin(d, x, y, z0) || x >= d.nx || y >= d.ny) return;
  const int z1 = min(z0 + TV_ZB, d.nz);
  const float* px = p;
  const float* py = p + d.nv;
  const float* pz = p + 2 * d.nv;
  const bool nxt_x = x + 1 < d.nx, prv_x = x >= 1;
  const bool nxt_y = y + 1 < d.ny, prv_y = y >= 1;
  size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
  float pz_prev = z0 >= 1 ? pz[v - d.plane] : 0.0f;
  for (int z = z0; z < z1; ++z, v += d.plane) {
    const float cz = pz[v];
    float r = 0.0f;
    if (nxt_x) r += px[v];
    if (prv_x) r -= px[v - 1];
    if (nxt_y) r += py[v];
    if (prv_y) r -= py[v - d.nx];
    if (z + 1 < d.nz) r += cz;
    if (z >= 1) r -= pz_prev;
    out[v] = r;
    pz_prev = cz;
  }
}

// out = base + rho * (-div)(grad mu - shift), i.e. the gradient of
// rho/2 ||grad mu - shift||^2 added to base (eq:gradtomo with
// shift = psi - lambda / rho).  base and shift may be NULL (zero).  With
// REDUCE the block also sums <out - g_old, eta> and ||out||^2 (out may
// alias g_old: each voxel is read before it is written by the same thread).
template <bool REDUCE>
__global__ __launch_bounds__(TV_NT) void k_tv_term(const float* __restrict__ mu,
                                                    const float* __restrict__ shift,
                                                    const float* base, float rho, float* out,
                                                    const float* g_old,
                                                    const float* __restrict__ eta,
                                                    double* __restrict__ partials, Vol3 d) {
  int x, y, z0;
  double s_dy = 0.0, s_gg = 0.0;
  const bool live = tile_origin(d, x, y, z0) && x < d.nx && y < d.ny;
  if (live) {
    const int z1 = min(z0 + TV_ZB, d.nz);
    const bool nxt_x = x + 1 < d.nx, prv_x = x >= 1;
    const bool nxt_y = y + 1 < d.ny, prv_y = y >= 1;
    const float* sx = shift;
    const float* sy = shift ? shift + d.nv : nullptr;
    const float* sz = shift ? shift + 2 * d.nv : nullptr;
    size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
    float m_prev = z0 >= 1 ? mu[v - d.plane] : 0.0f;
    float sz_prev = (z0 >= 1 && shift) ? sz[v - d.plane] : 0.0f;
    float m_c = mu[v];
    for (int z = z0; z < z1; ++z, v += d.plane) {
      const bool nxt_z = z + 1 < d.nz, prv_z = z >= 1;
      const float m_n = nxt_z ? mu[v + d.plane] : 0.0f;
      float t = 0.0f;
      // q_e(v) = mu(v + e) - mu(v) - s_e(v) enters with a minus sign where
      // v + e exists, q_e(v - e) with a plus sign where v - e exists.
      if (nxt_x) t -= (mu[v + 1] - m_c) - (shift ? sx[v] : 0.0f);
      if (prv_x) t += (m_c - mu[v - 1]) - (shift ? sx[v - 1] : 0.0f);
      if (nxt_y) t -= (mu[v + d.nx] - m_c) - (shift ? sy[v] : 0.0f);
      if (prv_y) t += (m_c - mu[v - d.nx]) - (shift ? sy[v - d.nx] : 0.0f);
      const float sz_c = shift ? sz[v] : 0.0f;
      if (nxt_z) t -= (m_n - m_c) - sz_c;
      if (prv_z) t += (m_c - m_prev) - sz_prev;
      const float r = (base ? base[v] : 0.0f) + rho * t;
      if (REDUCE) {
        const double go = g_old[v];
        s_dy += ((double)r - go) * (double)eta[v];
        s_gg += (double)r * (double)r;
      }
      out[v] = r;
      m_prev = m_c;
      m_c = m_n;
      sz_prev = sz_c;
    }
  }
  if (REDUCE) block_sum2(s_dy, s_gg, partials);
}

// psi = shrink(grad mu + lambda / rho, alpha / rho); lambda += rho (grad mu - psi);
// shift = psi - lambda / rho.  lambda is updated in place; psi_out may be NULL.
__global__ __launch_bounds__(TV_NT) void k_tv_shrink(const float* __restrict__ mu,
                                                      float* __restrict__ lam,
                                                      float* __restrict__ shift,
                                                      float* __restrict__ psi_out, float alpha,
                                                      float rho, Vol3 d) {
  int x, y, z0;
  if (!tile_origin(d, x, y, z0) || x >= d.nx || y >= d.ny) return;
  const int z1 = min(z0 + TV_ZB, d.nz);
  const size_t ox = x + 1 < d.nx ? 1 : 0;
  const size_t oy = y + 1 < d.ny ? d.nx : 0;
  const float inv_rho = 1.0f / rho;
  const float thr = alpha / rho;
  size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
  float c = mu[v];
  for (int z = z0; z < z1; ++z, v += d.plane) {
    const size_t oz = z + 1 < d.nz ? d.plane : 0;
    const float az = mu[v + oz];
    const float g[3] = {mu[v + ox] - c, mu[v + oy] - c, az - c};
    float l[3], q[3];
    float m2 = 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      l[k] = lam[v + k * d.nv];
      q[k] = g[k] + l[k] * inv_rho;
      m2 += q[k] * q[k];
    }
    const float mag = sqrtf(m2);
    const float sc = mag > thr ? 1.0f - thr / mag : 0.0f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ps = sc * q[k];
      const float ln = l[k] + rho * (g[k] - ps);
      lam[v + k * d.nv] = ln;
      shift[v + k * d.nv] = ps - ln * inv_rho;
      if (psi_out) psi_out[v + k * d.nv] = ps;
    }
    c = az;
  }
}

// ---------------------------------------------------------------------------
// Conjugate-gradient steps of the tomography sub-problem (Eq:tomo): the
// Dai-Yuan direction (Eq:DaiYuan2) with the exact line search of a
// quadratic.  Scalars live in S[]:
enum { S_GDOT = 0, S_GAMMA = 1, S_BETA = 2, S_STOP = 3, S_COUNT = 8 };

// eta = -g + beta eta (beta = 0 on a restart); partial sums of <g, eta>.
__global__ __launch_bounds__(TV_NT) void k_cg_dir(const float* __restrict__ g,
                                                   float* __restrict__ eta,
                                                   const double* __restrict__ S, int restart,
                                                   double* __restrict__ partials, Vol3 d) {
  int x, y, z0;
  double s = 0.0;
  if (tile_origin(d, x, y, z0) && x < d.nx && y < d.ny) {
    const float beta = restart ? 0.0f : (float)S[S_BETA];
    const int z1 = min(z0 + TV_ZB, d.nz);
    size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
    for (int z = z0; z < z1; ++z, v += d.plane) {
      const float gv = g[v];
      const float e = restart ? -gv : -gv + beta * eta[v];
      eta[v] = e;
      s += (double)gv * (double)e;
    }
  }
  block_sum2(s, 0.0, partials);
}

// Partial sums of ||grad eta||^2 (second slot; the first is 0).
__global__ __launch_bounds__(TV_NT) void k_cg_curv(const float* __restrict__ eta,
                                                    double* __restrict__ partials, Vol3 d) {
  int x, y, z0;
  double s_gr = 0.0;
  if (tile_origin(d, x, y, z0) && x < d.nx && y < d.ny) {
    const int z1 = min(z0 + TV_ZB, d.nz);
    const size_t ox = x + 1 < d.nx ? 1 : 0;
    const size_t oy = y + 1 < d.ny ? d.nx : 0;
    size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
    float c = eta[v];
    for (int z = z0; z < z1; ++z, v += d.plane) {
      const size_t oz = z + 1 < d.nz ? d.plane : 0;
      const float az = eta[v + oz];
      const float gx = eta[v + ox] - c, gy = eta[v + oy] - c, gz = az - c;
      s_gr += (double)gx * gx + (double)gy * gy + (double)gz * gz;
      c = az;
    }
  }
  block_sum2(0.0, s_gr, partials);
}

// Partial sums of ||q||^2 over a data array (q = L eta): the first slot of
// partials[2 * block], grid-stride over n values, float4 loads where aligned.
constexpr int SQ_BLOCKS = 1024;
__global__ __launch_bounds__(TV_NT) void k_sumsq(const float* __restrict__ q, size_t n,
                                                  double* __restrict__ partials) {
  double s = 0.0;
  const size_t n4 = n / 4;
  const float4* q4 = reinterpret_cast<const float4*>(q);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 v = q4[i];
    s += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    s += (double)q[i] * q[i];
  block_sum2(s, 0.0, partials);
}

// mu += gamma eta; w += gamma t  (w = L*(L mu - d) follows mu).
__global__ __launch_bounds__(TV_NT) void k_cg_step(float* __restrict__ mu,
                                                    const float* __restrict__ eta,
                                                    float* __restrict__ w,
                                                    const float* __restrict__ t,
                                                    const double* __restrict__ S, Vol3 d) {
  int x, y, z0;
  if (!tile_origin(d, x, y, z0) || x >= d.nx || y >= d.ny) return;
  const float gam = (float)S[S_GAMMA];
  const int z1 = min(z0 + TV_ZB, d.nz);
  size_t v = ((size_t)z0 * d.ny + y) * d.nx + x;
  for (int z = z0; z < z1; ++z, v += d.plane) {
    mu[v] += gam * eta[v];
    w[v] += gam * t[v];
  }
}

enum { FIN_GDOT = 0, FIN_GAMMA = 1, FIN_BETA = 2 };

// Sum the per-block partials in a fixed order and derive the CG scalars.
//   FIN_GDOT : S_GDOT = <g, eta>                (restart clears S_STOP)
//   FIN_GAMMA: gamma = -<g, eta> / (||L eta||^2 + rho ||grad eta||^2), the
//              first sum from the data-space partials p2 (n2 blocks)
//   FIN_BETA : beta = ||g_new||^2 / <g_new - g, eta>
// A zero denominator stops the sub-problem: gamma and beta stay 0 until
// the next restart, so mu no longer moves.
__global__ __launch_bounds__(TV_FIN) void k_cg_finalize(const double* __restrict__ partials,
                                                         int nblocks,
                                                         const double* __restrict__ p2, int n2,
                                                         double* __restrict__ S, int mode,
                                                         int restart, double rho) {
  __shared__ double r0[TV_FIN], r1[TV_FIN];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += TV_FIN) {
    a += partials[2 * i];
    b += partials[2 * i + 1];
  }
  for (int i = threadIdx.x; i < n2; i += TV_FIN) a += p2[2 * i];
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int s = TV_FIN / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      r0[threadIdx.x] += r0[threadIdx.x + s];
      r1[threadIdx.x] += r1[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  a = r0[0];
  b = r1[0];
  if (mode == FIN_GDOT) {
    S[S_GDOT] = a;
    if (restart) S[S_STOP] = 0.0;
  } else if (mode == FIN_GAMMA) {
    const double den = a + rho * b;
    const bool stop = S[S_STOP] != 0.0 || den == 0.0;
    S[S_GAMMA] = stop ? 0.0 : -S[S_GDOT] / den;
    if (stop) S[S_STOP] = 1.0;
  } else {
    const bool stop = S[S_STOP] != 0.0 || a == 0.0;
    S[S_BETA] = stop ? 0.0 : b / a;
    if (stop) S[S_STOP] = 1.0;
  }
}

__global__ void k_sub_inplace(float* __restrict__ q, const float* __restrict__ dd, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    q[i] -= dd[i];
}

__global__ void k_fill_zero(float* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = 0.0f;
}

int flat_blocks(size_t n) {
  const size_t b = (n + 255) / 256;
  return (int)(b < 8192 ? (b > 0 ? b : 1) : 8192);
}

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Layout of the caller's ADMM state buffer (bytes, each part 256-aligned):
//   lambda [3][nz][n][n] f32 | shift [3][nz][n][n] f32 | w, g, eta, t
//   [nz][n][n] f32 each | q [n_theta][h][w] f32 | volume partials f64 |
//   data partials f64 | scalars f64
struct AdmmLayout {
  size_t lam, shift, w, g, eta, t, q, partials, partials_q, scalars, total;
};

static AdmmLayout admm_layout(const lamino_plan_s* p) {
  const Vol3 d = vol3(p->nz, p->n, p->n);
  const size_t v4 = d.nv * 4;
  AdmmLayout L;
  size_t o = 0;
  L.lam = o;      o += a256(3 * v4);
  L.shift = o;    o += a256(3 * v4);
  L.w = o;        o += a256(v4);
  L.g = o;        o += a256(v4);
  L.eta = o;      o += a256(v4);
  L.t = o;        o += a256(v4);
  L.q = o;        o += a256((size_t)p->n_theta * p->h * p->w * 4);
  L.partials = o; o += a256((size_t)d.grid * 2 * 8);
  L.partials_q = o; o += a256((size_t)SQ_BLOCKS * 2 * 8);
  L.scalars = o;  o += a256(S_COUNT * 8);
  L.total = o;
  return L;
}

size_t admm_state_bytes(const lamino_plan_s* p) { return admm_layout(p).total; }

// The tile count must fit the launch grid (int) with room for the XCD padding.
bool tv_dims_ok(int nz, int ny, int nx) {
  if (nz <= 0 || ny <= 0 || nx <= 0) return false;
  const long long nb = (long long)((nx + TV_BX - 1) / TV_BX) * ((ny + TV_BY - 1) / TV_BY) *
                       ((nz + TV_ZB - 1) / TV_ZB);
  return nb <= (1LL << 30);
}

hipError_t tv_grad(const float* mu, float* out, int nz, int ny, int nx, hipStream_t s) {
  const Vol3 d = vol3(nz, ny, nx);
  hipLaunchKernelGGL(k_tv_grad, dim3(d.grid), dim3(TV_NT), 0, s, mu, out, d);
  return hipGetLastError();
}

hipError_t tv_div(const float* p, float* out, int nz, int ny, int nx, hipStream_t s) {
  const Vol3 d = vol3(nz, ny, nx);
  hipLaunchKernelGGL(k_tv_div, dim3(d.grid), dim3(TV_NT), 0, s, p, out, d);
  return hipGetLastError();
}

hipError_t tv_term(const float* mu, const float* shift, const float* base, float rho, float* out,
                   int nz, int ny, int nx, hipStream_t s) {
  const Vol3 d = vol3(nz, ny, nx);
  hipLaunchKernelGGL((k_tv_term<false>), dim3(d.grid), dim3(TV_NT), 0, s, mu, shift, base, rho,
                     out, (const float*)nullptr, (const float*)nullptr, (double*)nullptr, d);
  return hipGetLastError();
}

hipError_t tv_shrink(const float* mu, float* lam, float* shift, float* psi, float alpha, float rho,
                     int nz, int ny, int nx, hipStream_t s) {
  const Vol3 d = vol3(nz, ny, nx);
  hipLaunchKernelGGL(k_tv_shrink, dim3(d.grid), dim3(TV_NT), 0, s, mu, lam, shift, psi, alpha, rho,
                     d);
  return hipGetLastError();
}

// Appendix A's ADMM on the caller's stream.  Per outer iteration:
//   g = w - rho div(grad mu - shift), eta = -g           (restart)
//   inner times: q = L eta, t = L* q, gamma, mu += gamma eta, w += gamma t,
//                g_new, beta, eta = -g_new + beta eta    (the last two skipped
//                on the final inner step, whose direction is never used)
//   lambda, shift from the soft threshold and the dual update.
// w = L*(L mu - d) is formed once (resume == 0) and then follows mu.
hipError_t run_admm_tv(const lamino_plan_s* p, const float* d_data, float* mu, float alpha,
                       float rho, int outer, int inner, int resume, void* state, hipStream_t s) {
  const Vol3 d = vol3(p->nz, p->n, p->n);
  const AdmmLayout L = admm_layout(p);
  unsigned char* base = static_cast<unsigned char*>(state);
  float* lam = reinterpret_cast<float*>(base + L.lam);
  float* shift = reinterpret_cast<float*>(base + L.shift);
  float* w = reinterpret_cast<float*>(base + L.w);
  float* g = reinterpret_cast<float*>(base + L.g);
  float* eta = reinterpret_cast<float*>(base + L.eta);
  float* t = reinterpret_cast<float*>(base + L.t);
  float* q = reinterpret_cast<float*>(base + L.q);
  double* part = reinterpret_cast<double*>(base + L.partials);
  double* part_q = reinterpret_cast<double*>(base + L.partials_q);
  const double* no_p = nullptr;
  double* S = reinterpret_cast<double*>(base + L.scalars);
  const size_t nd = (size_t)p->n_theta * p->h * p->w;
  const dim3 grid(d.grid), blk(TV_NT), one(1), fin(TV_FIN);
  hipError_t e;

  if (!resume) {
    hipLaunchKernelGGL(k_fill_zero, dim3(flat_blocks(3 * d.nv)), dim3(256), 0, s, lam, 3 * d.nv);
    hipLaunchKernelGGL(k_fill_zero, dim3(flat_blocks(3 * d.nv)), dim3(256), 0, s, shift, 3 * d.nv);
    if ((e = run_forward(p, mu, q, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_sub_inplace, dim3(flat_blocks(nd)), dim3(256), 0, s, q, d_data, nd);
    if ((e = run_backprojection(p, q, w, false, s)) != hipSuccess) return e;
  }
  for (int k = 0; k < outer; ++k) {
    if (inner > 0) {
      hipLaunchKernelGGL((k_tv_term<false>), grid, blk, 0, s, (const float*)mu,
                         (const float*)shift, (const float*)w, rho, g, (const float*)nullptr,
                         (const float*)nullptr, (double*)nullptr, d);
      hipLaunchKernelGGL(k_cg_dir, grid, blk, 0, s, (const float*)g, eta, (const double*)S, 1,
                         part, d);
      hipLaunchKernelGGL(k_cg_finalize, one, fin, 0, s, (const double*)part, d.grid, no_p, 0, S,
                         (int)FIN_GDOT, 1, (double)rho);
    }
    for (int m = 0; m < inner; ++m) {
      if ((e = run_forward(p, eta, q, s)) != hipSuccess) return e;
      if ((e = run_backprojection(p, q, t, false, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(k_sumsq, dim3(SQ_BLOCKS), blk, 0, s, (const float*)q, nd, part_q);
      hipLaunchKernelGGL(k_cg_curv, grid, blk, 0, s, (const float*)eta, part, d);
      hipLaunchKernelGGL(k_cg_finalize, one, fin, 0, s, (const double*)part, d.grid,
                         (const double*)part_q, SQ_BLOCKS, S, (int)FIN_GAMMA, 0, (double)rho);
      hipLaunchKernelGGL(k_cg_step, grid, blk, 0, s, mu, (const float*)eta, w, (const float*)t,
                         (const double*)S, d);
      if (m + 1 < inner) {
        hipLaunchKernelGGL((k_tv_term<true>), grid, blk, 0, s, (const float*)mu,
                           (const float*)shift, (const float*)w, rho, g, (const float*)g,
                           (const float*)eta, part, d);
        hipLaunchKernelGGL(k_cg_finalize, one, fin, 0, s, (const double*)part, d.grid, no_p, 0,
                           S, (int)FIN_BETA, 0, (double)rho);
        hipLaunchKernelGGL(k_cg_dir, grid, blk, 0, s, (const float*)g, eta, (const double*)S, 0,
                           part, d);
        hipLaunchKernelGGL(k_cg_finalize, one, fin, 0, s, (const double*)part, d.grid, no_p, 0,
                           S, (int)FIN_GDOT, 0, (double)rho);
      }
    }
    hipLaunchKernelGGL(k_tv_shrink, grid, blk, 0, s, (const float*)mu, lam, shift, (float*)nullptr,
                       alpha, rho, d);
  }
  return hipGetLastError();
}

}  // namespace lam
