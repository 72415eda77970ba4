// Direct discretisation of the backprojection: the O(N^3 N_theta) method
// that the Fourier route replaces (eq:adj and eq:recon as line integrals
// with linear interpolation).  Voxel-driven bilinear form:
//   L*_dir d (x) = sum_theta  bilinear(d_theta)(x.e_u + w/2, x.e_v + h/2),
// detector pixels outside h x w read as zero; FBP_dir filters the detector
// rows first.
//
//   dir_filter       two detector rows packed as one complex w_p-point FFT
//                    (column c at padded index (c - w/2) mod w_p), times the
//                    real, even transfer function W(m) / w_p, inverse FFT,
//                    cropped back to w; several row pairs per block when w_p
//                    is small.
//   dir_backproject  a 256-thread block owns a 16 x 16 (x, y) column of
//                    voxels over DB_Z consecutive z planes (each wavefront an
//                    8 x 8 patch).  Per angle the block stages the detector
//                    window its tile projects into in LDS (zeros off the
//                    detector), then every thread walks its z column: the
//                    detector column c0 and its weight are the same for the
//                    whole column (e_u has no x3 part) and the row coordinate
//                    grows by cos(phi) <= 1 per plane, so the thread keeps the
//                    column-interpolated values of the two rows around its
//                    tap and reads one new row (two LDS reads) per plane.
//                    Projected coordinates are formed in double precision
//                    once per angle and column; the row fraction then steps
//                    in float.
#include "lamino_common.h"
#include "lamino_device.h"
#include "lamino_internal.h"

namespace lam {
namespace {

// block tile 16 (x) x 16 (y) x DB_Z; each wavefront owns an 8 x 8 (x, y)
// patch, whose projection covers a compact detector window at every angle
constexpr int DB_X = 16, DB_Y = 16, DB_Z = 16, DB_NT = DB_X * DB_Y;

template <int LOGN>
__global__ __launch_bounds__(NTF) void k_dir_filter(KParams p, const void* __restrict__ data,
                                                     float* __restrict__ out, int rows, int pairs_per_block) {
  extern __shared__ float2 buf[];  // fft_capacity(w_p) values (launch size)
  const int wp = p.w_p, w = p.w;
  const int pair0 = blockIdx.x * pairs_per_block;
  const int npairs = min(pairs_per_block, (rows + 1) / 2 - pair0);
  lds_zero(buf, npairs * wp);
  __syncthreads();
  // the block's rows are contiguous in memory: row 2 j is the real part of
  // transform j, row 2 j + 1 its imaginary part
  const int row0 = 2 * pair0;
  const int nrows = min(2 * npairs, rows - row0);
  float* bf = reinterpret_cast<float*>(buf);
  const float iw = 1.f / (float)w;
  with_data(p.data_dtype, [&](auto ty) {
    stage_in<float>(
        nrows * w, [&](int e) { return ld_rt<decltype(ty)::value>(data, (size_t)row0 * w + e); },
        [&](int e, float v) {
          const int rr = div24(e, w, iw), c = e - rr * w;
          bf[2 * ((rr >> 1) * wp + ((c - w / 2) & (wp - 1))) + (rr & 1)] = v;
        });
  });
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_wp, npairs, p.tw, p.log2_twmax, false);
  for (int e = threadIdx.x; e < npairs * wp; e += NTF) {
    const float f = p.filt_dir[e & (wp - 1)];
    buf[e].x *= f;
    buf[e].y *= f;
  }
  __syncthreads();
  block_fft<LOGN>(buf, p.log2_wp, npairs, p.tw, p.log2_twmax, true);
  for (int e = threadIdx.x; e < nrows * w; e += NTF) {
    const int rr = div24(e, w, iw), c = e - rr * w;
    out[(size_t)row0 * w + e] = bf[2 * ((rr >> 1) * wp + ((c - w / 2) & (wp - 1))) + (rr & 1)];
  }
}

// One detector value through a buffer resource: a byte offset outside the
// resource reads 0 (the hardware range check), which is how rows above and
// below the detector drop out.
constexpr int kBufferDword3 = 0x00020000;  // gfx9-family raw buffer descriptor word 3
template <int DT>
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, int byte_off) {
  if constexpr (DT == LAMINO_F32)
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
  else if constexpr (DT == LAMINO_U8)
    return (float)__builtin_amdgcn_raw_buffer_load_b8(r, byte_off, 0, 0);
  else if constexpr (DT == LAMINO_U16)
    return (float)__builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0);
  else if constexpr (DT == LAMINO_F16)
    return __half2float(__builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0)));
  else
    return __bfloat162float(
        __builtin_bit_cast(__hip_bfloat16, __builtin_amdgcn_raw_buffer_load_b16(r, byte_off, 0, 0)));
}
template <int DT>
constexpr int elem_bytes() {
  return DT == LAMINO_F32 ? 4 : (DT == LAMINO_U8 ? 1 : 2);
}

// Backprojection: per angle the block copies the detector window its
// 16 x 16 x DB_Z tile projects into (plus a one-pixel margin, zeros outside
// the detector) into LDS and gathers the taps there.  The window of a tile
// spans at most 15 (|cos| + |sin|) + 4 <= 26 columns and
// 15 (|sin(phi)| sqrt(2) + |cos(phi)|) + 4 <= 31 rows, so a 32 x 32 buffer
// holds it for every angle and tilt; two buffers alternate between angles
// and the next angle's window is fetched into registers while the current
// one is in use.
constexpr int WIN = 32, WIN_LD = WIN + 1;  // padded row stride against bank conflicts
constexpr int WIN_PER_THREAD = WIN * WIN / DB_NT;

template <int DT>
__global__ __launch_bounds__(DB_NT) void k_dir_backproject(KParams p, const void* __restrict__ d,
                                                                float* __restrict__ vol, int nbx, int nby,
                                                                int nb, int grid) {
  constexpr int EB = elem_bytes<DT>();
  __shared__ float win[2][WIN * WIN_LD];
  int bx, by, bz;
  if (!xcd_tile(blockIdx.x, grid, nb, nbx, nby, bx, by, bz)) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int ix = bx * DB_X + (wv & 1) * 8 + (lane & 7);
  const int iy = by * DB_Y + (wv >> 1) * 8 + (lane >> 3);
  const int z0 = bz * DB_Z;
  const double x1 = ix - p.n / 2, x2 = iy - p.n / 2, x30 = z0 - p.nz / 2;
  // tile corners (uniform): x1 in [X0, X0 + 15], x2 in [Y0, Y0 + 15]
  const double X0 = bx * DB_X - p.n / 2, Y0 = by * DB_Y - p.n / 2;
  const double uc = p.w / 2, vc = p.h / 2;
  const double sphi = p.sin_phi, cphid = p.cos_phi;
  const float cphi = (float)cphid;
  const int w = p.w;
  const size_t plane = (size_t)p.h * w;
  const double zspan = (DB_Z - 1) * cphid;

  // window origin of angle t (uniform)
  auto origin = [&](int t, int& r_lo, int& c_lo) {
    const double2 cs = p.trig_d[t];
    const double u0 = X0 * cs.x + Y0 * cs.y + uc;
    const double du = fmin(0.0, (DB_X - 1) * cs.x) + fmin(0.0, (DB_Y - 1) * cs.y);
    const double v0 = (X0 * cs.y - Y0 * cs.x) * sphi + x30 * cphid + vc;
    const double dv = (fmin(0.0, (DB_X - 1) * cs.y * sphi) + fmin(0.0, -(DB_Y - 1) * cs.x * sphi)) +
                      fmin(0.0, zspan);
    c_lo = (int)floor(u0 + du) - 1;
    r_lo = (int)floor(v0 + dv) - 1;
  };
  // this thread's share of angle t's window, zeros off the detector
  auto fetch = [&](int t, int r_lo, int c_lo, float (&v)[WIN_PER_THREAD]) {
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(static_cast<const char*>(d)) + (size_t)t * plane * EB, (short)0,
        (int)(plane * EB), kBufferDword3);
#pragma unroll
    for (int i = 0; i < WIN_PER_THREAD; ++i) {
      const int e = i * DB_NT + (int)threadIdx.x;
      const int c = c_lo + (e & (WIN - 1)), r = r_lo + e / WIN;
      const int cc = min(max(c, 0), w - 1);
      const float x = bload<DT>(rsrc, __mul24(r, w * EB) + EB * cc);  // rows outside read 0
      v[i] = (unsigned)c < (unsigned)w ? x : 0.f;
    }
  };
  auto place = [&](int buf, const float (&v)[WIN_PER_THREAD]) {
#pragma unroll
    for (int i = 0; i < WIN_PER_THREAD; ++i) {
      const int e = i * DB_NT + (int)threadIdx.x;
      win[buf][(e / WIN) * WIN_LD + (e & (WIN - 1))] = v[i];
    }
  };

  float acc[DB_Z];
#pragma unroll
  for (int k = 0; k < DB_Z; ++k) acc[k] = 0.f;
  float nxt[WIN_PER_THREAD];
  int r_lo, c_lo;
  origin(0, r_lo, c_lo);
  fetch(0, r_lo, c_lo, nxt);
  for (int t = 0; t < p.n_theta; ++t) {
    const int buf = t & 1;
    place(buf, nxt);
    __syncthreads();
    const int wr0 = r_lo, wc0 = c_lo;
    if (t + 1 < p.n_theta) {
      origin(t + 1, r_lo, c_lo);
      fetch(t + 1, r_lo, c_lo, nxt);
    }
    const double2 cs = p.trig_d[t];
    const double cc = fma(x1, cs.x, x2 * cs.y) + uc;
    const double rs = fma(fma(x1, cs.y, -x2 * cs.x), sphi, fma(x30, cphid, vc));
    const double c0d = floor(cc), r0d = floor(rs);
    const int cw = (int)c0d - wc0;  // window column of the left tap
    int rw = (int)r0d - wr0;        // window row of the upper tap
    float f = (float)(rs - r0d);
    const float fc = (float)(cc - c0d);
    const float* wb = win[buf] + cw;
    auto rowv = [&](int r) {
      const float* q = wb + r * WIN_LD;
      return q[0] + fc * (q[1] - q[0]);
    };
    float hcur = rowv(rw), hnext = rowv(rw + 1);
#pragma unroll
    for (int k = 0; k < DB_Z; ++k) {
      if (k > 0) {
        f += cphi;
        const bool adv = f >= 1.f;
        f = adv ? f - 1.f : f;
        rw += adv ? 1 : 0;
        const float hn = rowv(rw + 1);
        hcur = adv ? hnext : hcur;
        hnext = hn;
      }
      acc[k] += hcur + f * (hnext - hcur);
    }
  }
  if (ix >= p.n || iy >= p.n) return;
  size_t v = ((size_t)z0 * p.n + iy) * p.n + ix;
  const size_t vplane = (size_t)p.n * p.n;
#pragma unroll
  for (int k = 0; k < DB_Z; ++k, v += vplane)
    if (z0 + k < p.nz) vol[v] = acc[k];
}

}  // namespace

size_t direct_work_bytes(const lamino_plan_s* p) {
  return ((size_t)p->n_theta * p->h * p->w * 4 + 255) & ~(size_t)255;
}

hipError_t run_direct(const lamino_plan_s* p, const void* d_data, float* d_vol, void* d_work,
                      bool fbp_filter, hipStream_t s) {
  KParams kp = make_params(p, true);
  const void* src = d_data;
  int dt = p->opts.data_dtype;
  if (fbp_filter) {
    const int rows = p->n_theta * p->h;
    const int pairs = (rows + 1) / 2;
    const int ppb = std::max(1, std::min(fft_capacity(p->w_p) / p->w_p, 16));
    hipLaunchKernelGGL((p->w_p > LDS_CPLX ? k_dir_filter<13> : k_dir_filter<0>), dim3((pairs + ppb - 1) / ppb), dim3(NTF),
                       (size_t)fft_capacity(p->w_p) * sizeof(float2), s, kp, d_data,
                       static_cast<float*>(d_work), rows, ppb);
    src = d_work;
    dt = LAMINO_F32;
  }
  const int nbx = (p->n + DB_X - 1) / DB_X, nby = (p->n + DB_Y - 1) / DB_Y;
  const int nbz = (p->nz + DB_Z - 1) / DB_Z;
  const int nb = nbx * nby * nbz, grid = 8 * ((nb + 7) / 8);
  if (dt == LAMINO_F32)
    hipLaunchKernelGGL(k_dir_backproject<LAMINO_F32>, dim3(grid), dim3(DB_NT), 0, s, kp, src, d_vol,
                       nbx, nby, nb, grid);
  else if (dt == LAMINO_F16)
    hipLaunchKernelGGL(k_dir_backproject<LAMINO_F16>, dim3(grid), dim3(DB_NT), 0, s, kp, src, d_vol,
                       nbx, nby, nb, grid);
  else if (dt == LAMINO_BF16)
    hipLaunchKernelGGL(k_dir_backproject<LAMINO_BF16>, dim3(grid), dim3(DB_NT), 0, s, kp, src, d_vol,
                       nbx, nby, nb, grid);
  else if (dt == LAMINO_U16)
    hipLaunchKernelGGL(k_dir_backproject<LAMINO_U16>, dim3(grid), dim3(DB_NT), 0, s, kp, src, d_vol,
                       nbx, nby, nb, grid);
  else
    hipLaunchKernelGGL(k_dir_backproject<LAMINO_U8>, dim3(grid), dim3(DB_NT), 0, s, kp, src, d_vol,
                       nbx, nby, nb, grid);
  return hipGetLastError();
}

}  // namespace lam
