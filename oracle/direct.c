/* O1: direct discretisation of the line integrals with linear
 * interpolation (oracle, test infrastructure only; FP64, OpenMP).
 *
 * The paper contrasts the Fourier route with a direct discretisation of
 * eq:fwd and eq:adj using linear interpolation, costing O(N^3 N_theta)
 * (Section "Laminography reconstruction", the paragraph after the filter
 * description).  The form used here is voxel-driven:
 *
 *   L_dir f(t, r, c) = sum_x f(x) hat(u_c - x.e_u) hat(v_r - x.e_v)
 *   L*_dir d(x)      = sum_t sum_{r,c} d(t, r, c) hat(u_c - x.e_u) hat(v_r - x.e_v)
 *
 * with hat(s) = max(0, 1 - |s|), u_c = c - w/2 (integer division),
 * v_r = r - h/2, x1 = ix - n/2, x2 = iy - n/2, x3 = iz - nz/2, and e_u, e_v
 * read off the two deltas of eq:fwd:
 *   e_u = (cos t, sin t, 0),  e_v = (sin t sin p, -cos t sin p, cos p).
 * Pixels outside the h x w detector are dropped, so the pair is an exact
 * transpose.  Array layouts: f[iz][iy][ix], d[t][r][c], row-major.
 */
#include <math.h>
#include <stddef.h>

static void axes(double t, double p, double eu[3], double ev[3]) {
  eu[0] = cos(t);
  eu[1] = sin(t);
  eu[2] = 0.0;
  ev[0] = sin(t) * sin(p);
  ev[1] = -cos(t) * sin(p);
  ev[2] = cos(p);
}

void lam_direct_fwd(const double* f, int nz, int n, const double* theta,
                    int n_theta, double phi, int h, int w, double* d) {
  #pragma omp parallel for schedule(dynamic, 1)
  for (int t = 0; t < n_theta; ++t) {
    double eu[3], ev[3];
    axes(theta[t], phi, eu, ev);
    double* dt = d + (size_t)t * h * w;
    for (size_t i = 0; i < (size_t)h * w; ++i) dt[i] = 0.0;
    for (int iz = 0; iz < nz; ++iz) {
      const double x3 = iz - nz / 2;
      for (int iy = 0; iy < n; ++iy) {
        const double x2 = iy - n / 2;
        for (int ix = 0; ix < n; ++ix) {
          const double val = f[((size_t)iz * n + iy) * n + ix];
          if (val == 0.0) continue;
          const double x1 = ix - n / 2;
          const double pu = x1 * eu[0] + x2 * eu[1] + x3 * eu[2];
          const double pv = x1 * ev[0] + x2 * ev[1] + x3 * ev[2];
          const double cc = pu + w / 2, rr = pv + h / 2;
          const double c0f = floor(cc), r0f = floor(rr);
          const int c0 = (int)c0f, r0 = (int)r0f;
          const double fc = cc - c0f, fr = rr - r0f;
          for (int a = 0; a < 2; ++a) {
            const int r = r0 + a;
            if (r < 0 || r >= h) continue;
            const double wr = a ? fr : 1.0 - fr;
            for (int b = 0; b < 2; ++b) {
              const int c = c0 + b;
              if (c < 0 || c >= w) continue;
              const double wc = b ? fc : 1.0 - fc;
              dt[(size_t)r * w + c] += val * wr * wc;
            }
          }
        }
      }
    }
  }
}

void lam_direct_adj(const double* d, int nz, int n, const double* theta,
                    int n_theta, double phi, int h, int w, double* f) {
  #pragma omp parallel for collapse(2) schedule(static)
  for (int iz = 0; iz < nz; ++iz) {
    for (int iy = 0; iy < n; ++iy) {
      const double x3 = iz - nz / 2;
      const double x2 = iy - n / 2;
      for (int ix = 0; ix < n; ++ix) {
        const double x1 = ix - n / 2;
        double acc = 0.0;
        for (int t = 0; t < n_theta; ++t) {
          double eu[3], ev[3];
          axes(theta[t], phi, eu, ev);
          const double pu = x1 * eu[0] + x2 * eu[1] + x3 * eu[2];
          const double pv = x1 * ev[0] + x2 * ev[1] + x3 * ev[2];
          const double cc = pu + w / 2, rr = pv + h / 2;
          const double c0f = floor(cc), r0f = floor(rr);
          const int c0 = (int)c0f, r0 = (int)r0f;
          const double fc = cc - c0f, fr = rr - r0f;
          const double* dt = d + (size_t)t * h * w;
          for (int a = 0; a < 2; ++a) {
            const int r = r0 + a;
            if (r < 0 || r >= h) continue;
            const double wr = a ? fr : 1.0 - fr;
            for (int b = 0; b < 2; ++b) {
              const int c = c0 + b;
              if (c < 0 || c >= w) continue;
              const double wc = b ? fc : 1.0 - fc;
              acc += dt[(size_t)r * w + c] * wr * wc;
            }
          }
        }
        f[((size_t)iz * n + iy) * n + ix] = acc;
      }
    }
  }
}

/* Adjoint restricted to z-slices [z0, z1): used to time the direct method
 * on a bounded sample of a large volume. Writes f[(iz - z0)][iy][ix]. */
void lam_direct_adj_slices(const double* d, int nz, int n, const double* theta,
                           int n_theta, double phi, int h, int w, int z0,
                           int z1, double* f) {
  #pragma omp parallel for collapse(2) schedule(static)
  for (int iz = z0; iz < z1; ++iz) {
    for (int iy = 0; iy < n; ++iy) {
      const double x3 = iz - nz / 2;
      const double x2 = iy - n / 2;
      for (int ix = 0; ix < n; ++ix) {
        const double x1 = ix - n / 2;
        double acc = 0.0;
        for (int t = 0; t < n_theta; ++t) {
          double eu[3], ev[3];
          axes(theta[t], phi, eu, ev);
          const double pu = x1 * eu[0] + x2 * eu[1] + x3 * eu[2];
          const double pv = x1 * ev[0] + x2 * ev[1] + x3 * ev[2];
          const double cc = pu + w / 2, rr = pv + h / 2;
          const double c0f = floor(cc), r0f = floor(rr);
          const int c0 = (int)c0f, r0 = (int)r0f;
          const double fc = cc - c0f, fr = rr - r0f;
          const double* dt = d + (size_t)t * h * w;
          for (int a = 0; a < 2; ++a) {
            const int r = r0 + a;
            if (r < 0 || r >= h) continue;
            const double wr = a ? fr : 1.0 - fr;
            for (int b = 0; b < 2; ++b) {
              const int c = c0 + b;
              if (c < 0 || c >= w) continue;
              const double wc = b ? fc : 1.0 - fc;
              acc += dt[(size_t)r * w + c] * wr * wc;
            }
          }
        }
        f[((size_t)(iz - z0) * n + iy) * n + ix] = acc;
      }
    }
  }
}
