/* lamino.h -- C ABI of the MI355X laminography library.
 *
 * The library evaluates the laminographic projection L (eq:fwd), its
 * adjoint L* (eq:adj) and the filtered backprojection W L* (eq:recon) by
 * the Fourier route of the paper (eq:fftfwd, eq:fftadj): a 2D FFT per
 * projection, a Gaussian unequally-spaced FFT onto the tilted frequency
 * grid of eq:uneqspace, split as in eq:fftfwdsplit into per-slab 2D
 * transforms and a transform along x3.
 *
 * Conventions (all sizes in elements, all arrays C-order, row-major):
 *   volume  vol[nz][n][n], float32, x1 = ix - n/2 fastest, then
 *           x2 = iy - n/2, x3 = iz - nz/2 (integer division), voxel = 1;
 *   data    d[n_theta][h][w] in opts.data_dtype, detector column
 *           u = c - w/2 fastest, row v = r - h/2, pixel = 1;
 *   angles  theta_j (radians, any values; default 2 pi j / n_theta);
 *   tilt    phi in radians, 0 == tomography, |phi| < pi/2.
 * The detector is zero-padded to h_p x w_p (powers of two >= pad * (h, w));
 * frequencies are m / w_p and l / h_p without the Nyquist bins.  Under
 * these conventions lamino_fwd and lamino_adj are an exact adjoint pair
 * (up to rounding and the USFFT kernel truncation, which both share), and
 * lamino_fbp applies W(m) = (pi / n_theta) cos(phi) |m / w_p| window(m / w_p)
 * before backprojection (the Jacobian of eq:uneqspace and the double cover
 * of xi by theta in [0, 2 pi)).
 *
 * Memory ownership: the library never allocates device memory.  The caller
 * allocates the table and workspace buffers whose sizes lamino_plan_sizes
 * reports, binds them once with lamino_plan_bind, and passes input and
 * output device buffers to each call.  A plan with its workspace serves
 * one call at a time; concurrent calls need separate plans/workspaces.
 *
 * Streams: every call is asynchronous on the given HIP stream
 * (hipStream_t passed as void*; NULL = the default stream).  Results are
 * ready when the stream is synchronised.
 *
 * Errors: functions return LAMINO_OK (0) or a negative code; no call
 * throws.  lamino_last_error() gives a thread-local message for the last
 * failure on the calling thread.
 */
#ifndef LAMINO_H
#define LAMINO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lamino_plan_s lamino_plan_t;

/* Element types.  LAMINO_U8 and LAMINO_U16 (8- and 16-bit detector values,
 * read as floats) are accepted for input data only: lamino_fwd rejects a
 * plan with integer data. */
typedef enum {
  LAMINO_F32 = 0,
  LAMINO_F16 = 1,
  LAMINO_BF16 = 2,
  LAMINO_U8 = 3,
  LAMINO_U16 = 4
} lamino_dtype;

/* Window of the FBP filter (the paper names ramp, Shepp-Logan, Parzen). */
typedef enum { LAMINO_RAMP = 0, LAMINO_SHEPP_LOGAN = 1, LAMINO_PARZEN = 2 } lamino_filter;

enum {
  LAMINO_OK = 0,
  LAMINO_E_INVALID = -1,     /* bad argument: sizes, tilt, NULL pointer */
  LAMINO_E_UNSUPPORTED = -2, /* size outside what the kernels support   */
  LAMINO_E_BUDGET = -3,      /* workspace exceeds opts.hbm_budget        */
  LAMINO_E_HIP = -4,         /* HIP runtime or launch error              */
  LAMINO_E_UNBOUND = -5      /* plan used before lamino_plan_bind        */
};

/* Scan geometry (eq:fwd).  theta is a host array of n_theta radians or
 * NULL for 2 pi j / n_theta; it is copied by lamino_plan. */
typedef struct {
  int nz, n;       /* volume nz x n x n                         */
  int n_theta;     /* number of projections                     */
  int h, w;        /* detector rows x columns                   */
  double tilt;     /* phi (radians)                             */
  const double* theta;
} lamino_geom;

/* Options; zero-initialise and then call lamino_opts_default. */
typedef struct {
  int data_dtype;     /* lamino_dtype of d (F32, F16, BF16; U8, U16 input only) */
  int storage_dtype;  /* lamino_dtype of the stored spectra and slab planes.
                         Accumulation is float32 throughout.  Gridding and
                         the x3 transform multiply on the matrix cores: with
                         float32 storage each operand is split into bfloat16
                         hi + lo parts (three products, ~2^-17 relative
                         error); float16 / bfloat16 storage multiplies the
                         stored values directly                               */
  int filter;         /* lamino_filter used by lamino_fbp                      */
  double pad_u, pad_v;/* detector padding factors (>= 1), default 2           */
  int kernel_m;       /* Gaussian half-width M in grid cells (2..8); 0 picks
                         5 for F32 storage and 3 for F16/BF16 storage          */
  int z_chunk;        /* x3-transform output slices per launch; 0 = nz         */
  int slab_chunk;     /* frequency slabs gridded per pass; 0 = automatic       */
  int theta_chunk;    /* projections per detector-FFT pass; 0 = automatic      */
  size_t hbm_budget;  /* max workspace bytes; 0 = no limit.  Chunks shrink to
                         fit; if the device-resident workspace still exceeds
                         the budget, the slab planes g and then also the
                         spectra D are kept in a caller-owned host buffer
                         (lamino_plan_host_sizes / lamino_plan_bind_host)
                         and streamed through double-buffered device chunks */
} lamino_opts;

/* Derived sizes of a plan (read-only description). */
typedef struct {
  int h_p, w_p;       /* padded detector                                      */
  int n_slab;         /* stored frequency slabs l = 0 .. h_p/2 - 1             */
  int grid;           /* per-slab USFFT grid N_g: power of two >= max(32, 2n) */
  int kernel_m;       /* Gaussian half-width M                                */
  double beta;        /* Gaussian exponent: phi(t) = exp(-beta t^2), t in cells*/
  int z_chunk, slab_chunk, theta_chunk;
  size_t table_bytes, work_bytes;
  size_t off_spectra, bytes_spectra; /* D[l][theta][k] in the workspace       */
  size_t off_slabs, bytes_slabs;     /* g[l][y][x] in the workspace           */
  double spectra_scale; /* power of two by which the stored D and g of an
                           FBP exceed their definition: h_p w_p / 64 for F16
                           storage (keeps typical values out of the float16
                           subnormal range), else 1; the x3 transform removes
                           it.  With F16 storage L* uses spectra_scale /
                           2^ceil(log2 n_theta), the forward L carries
                           1 / 2^ceil(log2 nz) on g and 2^15 / 2^ceil(log2
                           32 n^2) on D, and every call also scales its input
                           by 2^-e so that its largest magnitude lies in
                           [0.5, 1) (a scan of the input, undone at the
                           output): float16 intermediates stay in range for
                           any input scale                                    */
  int spill_spectra;  /* 1: D lives in the host buffer (out-of-core plan)     */
  int spill_slabs;    /* 1: g lives in the host buffer                        */
  int col_chunk;      /* x3 columns per chunk when g lives in host memory     */
  int io_z;           /* volume slices per chunk of lamino_fbp_host           */
  size_t host_bytes;  /* host buffer bytes (0: everything on the device)      */
  size_t io_bytes;    /* device staging bytes of lamino_fbp_host              */
} lamino_info;

/* Fill *opts with defaults (F32 data and storage, Shepp-Logan, pad 2). */
void lamino_opts_default(lamino_opts* opts);

/* Create a plan for geometry *geom (host-only: no HIP call).  Computes the
 * per-angle trigonometry, the x3 phase table, the filter, the USFFT psi
 * correction and FFT twiddles in double precision and keeps them on the
 * host until bind.  opts may be NULL (defaults).  On success *out owns a
 * new plan.  Errors: E_INVALID (non-positive sizes, |tilt| >= pi/2,
 * non-finite values, NULL out), E_UNSUPPORTED (a padded size above 8192 or
 * a grid the FFT kernels do not cover), E_BUDGET (workspace > hbm_budget
 * even at the smallest chunks). */
int lamino_plan(const lamino_geom* geom, const lamino_opts* opts, lamino_plan_t** out);

/* Bytes of the device table buffer and the device workspace the caller
 * must provide to lamino_plan_bind (each 256-byte aligned).  Host-only. */
int lamino_plan_sizes(const lamino_plan_t* plan, size_t* table_bytes, size_t* work_bytes);

/* Derived sizes and workspace layout.  Host-only. */
int lamino_plan_info(const lamino_plan_t* plan, lamino_info* info);

/* Attach caller-owned device buffers (d_tables: table_bytes, d_work:
 * work_bytes, both 256-byte aligned) and upload the tables on `stream`.
 * The buffers must outlive every later call with this plan.  Rebinding is
 * allowed.  Errors: E_INVALID (NULL/misaligned buffers), E_HIP. */
int lamino_plan_bind(lamino_plan_t* plan, void* d_tables, void* d_work, void* stream);

/* Host memory of an out-of-core plan (Section "GPU acceleration of
 * reconstruction": chunks streamed between host and device memory on
 * separate streams, transfers overlapping compute).  *host_bytes: bytes of
 * the caller-owned host buffer that holds the spectra D[l][theta][k] and / or
 * the slab planes g[l][y][x] when the device workspace alone exceeds
 * opts.hbm_budget (0 for a device-resident plan).  *io_bytes: bytes of the
 * device staging buffer lamino_fbp_host needs (data and volume chunks).
 * Either pointer may be NULL.  Host-only. */
int lamino_plan_host_sizes(const lamino_plan_t* plan, size_t* host_bytes, size_t* io_bytes);

/* Attach the caller-owned host buffer of host_bytes bytes (256-byte
 * aligned; pinned memory, e.g. hipHostMalloc, for transfers that overlap
 * compute).  Required before any call on a plan with host_bytes > 0, and
 * must outlive those calls; no HIP call.  Errors: E_INVALID. */
int lamino_plan_bind_host(lamino_plan_t* plan, void* h_spill);

/* Copy the plan's table image (table_bytes bytes: the per-angle
 * trigonometry, filters, psi correction, x3 phases and twiddles computed in
 * double precision by lamino_plan) into caller host memory host_dst of
 * `bytes` >= table_bytes bytes, typically pinned memory from which the
 * caller uploads it asynchronously on its own stream.  Host-only.
 * Errors: E_INVALID (NULL argument, bytes too small). */
int lamino_plan_table_image(const lamino_plan_t* plan, void* host_dst, size_t bytes);

/* Attach caller-owned device buffers without uploading anything (no HIP
 * call): d_tables must hold this plan's table image by the time a later
 * call on the plan runs, e.g. through a copy from lamino_plan_table_image's
 * output enqueued earlier on the call's stream.  Same buffer rules as
 * lamino_plan_bind; this is the non-blocking form of binding for request
 * loops that re-bind one workspace to many plans.  Errors: E_INVALID. */
int lamino_plan_attach(lamino_plan_t* plan, void* d_tables, void* d_work);

/* Filtered backprojection (eq:recon via eq:fftadj): vol = L*(W d).
 * d_data: device d[n_theta][h][w] in data_dtype (read only);
 * d_vol: device float vol[nz][n][n] (written).  Errors: E_INVALID,
 * E_UNBOUND, E_HIP. */
int lamino_fbp(const lamino_plan_t* plan, const void* d_data, float* d_vol, void* stream);

/* Filtered backprojection with the data and the volume in host memory,
 * for volumes or inputs larger than the device can hold: projection chunks
 * (theta_chunk at a time) are copied in, the volume leaves in chunks of
 * io_z slices (or, when the plan keeps g in host memory, in column chunks
 * of all slices), each through two alternating device buffers of the
 * caller-owned staging buffer d_io (io_bytes, 256-byte aligned), with the
 * copies on two library-owned streams (default priority) overlapping the
 * kernels on `stream`.  h_data: host d[n_theta][h][w] in data_dtype;
 * h_vol: host float vol[nz][n][n] (written); both should be pinned.  The
 * results equal lamino_fbp's.  When the call's work on `stream` is
 * complete, h_vol is written.  With float16 storage the data are read
 * twice (a scan for the input factor, then the transforms).  Errors as
 * lamino_fbp. */
int lamino_fbp_host(const lamino_plan_t* plan, const void* h_data, float* h_vol, void* d_io,
                    void* stream);

/* Filtered backprojection of raw detector counts.  The recording model of
 * Section "Laminography reconstruction" (the paragraph after eq:fwd),
 * raw = exp(-d) (flat - dark) + dark, is inverted inside the first detector
 * kernel while it stages the data:
 *   d = -log(max(ratio, min_ratio)),  ratio = (raw - dark) / (flat - dark),
 * with ratio = min_ratio where flat - dark <= 0 (dead pixels); then as
 * lamino_fbp.  d_raw: device [n_theta][h][w] in the plan's data dtype
 * (typically U16 or U8); d_dark, d_flat: device float32 [h][w] (averaged
 * dark- and flat-field images); min_ratio > 0 (E_INVALID otherwise).
 * The corrected data are never written to memory.  Errors as lamino_fbp. */
int lamino_fbp_raw(const lamino_plan_t* plan, const void* d_raw, const float* d_dark,
                   const float* d_flat, double min_ratio, float* d_vol, void* stream);

/* Slices of the FBP with a rotation-axis offset: the axis sits at detector
 * column w/2 + center_shift (fractional allowed) instead of w/2, which in
 * the Fourier route is the phase ramp exp(2 pi i m center_shift / w_p) on
 * every row spectrum (a translation of the trigonometric interpolant of the
 * padded rows); only slices z_first .. z_first + z_count - 1 of the x3
 * transform are formed.  This is the single-slice reconstruction that the
 * axis and tilt searches of the paper repeat over a sweep (Section "Mouse
 * brain imaging"); a tilt sweep uses one plan per tilt (plans of one shape
 * may share a workspace when their calls do not overlap).
 * d_out: device float [z_count][n][n].  Errors: E_INVALID (slice range
 * outside [0, nz), |center_shift| > (w_p - w)/2 or not finite), E_UNBOUND,
 * E_HIP. */
int lamino_fbp_slices(const lamino_plan_t* plan, const void* d_data, double center_shift,
                      int z_first, int z_count, float* d_out, void* stream);

/* Forward projection (eq:fwd via eq:fftfwd): d = L vol.
 * d_vol: device float vol[nz][n][n] (read only); d_data: device
 * d[n_theta][h][w] in data_dtype (written; E_INVALID for integer data).
 * Errors as lamino_fbp, and E_UNSUPPORTED for an out-of-core plan. */
int lamino_fwd(const lamino_plan_t* plan, const float* d_vol, void* d_data, void* stream);

/* Adjoint (eq:adj via eq:fftadj): vol = L* d, the exact transpose of
 * lamino_fwd.  Arguments as lamino_fbp. */
int lamino_adj(const lamino_plan_t* plan, const void* d_data, float* d_vol, void* stream);

/* ---------------------------------------------------------------------
 * Direct discretisation (the O(N^3 N_theta) method the Fourier route
 * replaces: eq:adj and eq:recon evaluated as line integrals with linear
 * interpolation).  Voxel-driven bilinear form on the plan's geometry:
 *   L*_dir d (x) = sum_theta sum_{r,c} d(theta, r, c) hat(u_c - x.e_u) hat(v_r - x.e_v),
 *   hat(s) = max(0, 1 - |s|), u_c = c - w/2, v_r = r - h/2,
 * i.e. bilinear interpolation of each projection at (x.e_u, x.e_v) with
 * detector pixels outside h x w taken as zero.  FBP_dir first filters every
 * detector row with W(m) (the transfer function of lamino_fbp, including
 * (pi / n_theta) cos(phi)): rows zero-padded to w_p (column c at index
 * (c - w/2) mod w_p), w_p-point DFT, multiply, inverse DFT, cropped back to
 * w.  Arithmetic: float32 with projected coordinates formed in float64. */

/* Bytes of the workspace lamino_direct_fbp needs (the filtered rows:
 * n_theta * h * w float32, 256-byte multiple).  Host-only. */
int lamino_direct_work_bytes(const lamino_plan_t* plan, size_t* bytes);

/* vol = L*_dir (filtered d).  d_data: device d[n_theta][h][w] in the plan's
 * data dtype; d_vol: device float vol[nz][n][n] (written); d_work: device
 * buffer of lamino_direct_work_bytes bytes, 256-byte aligned (contents
 * overwritten).  Errors: E_INVALID, E_UNBOUND, E_HIP. */
int lamino_direct_fbp(const lamino_plan_t* plan, const void* d_data, float* d_vol, void* d_work,
                      void* stream);

/* vol = L*_dir d (no filter).  Arguments as lamino_direct_fbp without the
 * workspace. */
int lamino_direct_adj(const lamino_plan_t* plan, const void* d_data, float* d_vol, void* stream);

/* Stages reported by lamino_plan_stage_times. */
enum {
  LAMINO_STAGE_DETECTOR = 0, /* per-projection 2D FFTs and filter          */
  LAMINO_STAGE_GRIDDING = 1, /* USFFT spreading (L*, FBP) / interpolation (L) */
  LAMINO_STAGE_SLAB = 2,     /* per-slab 2D FFTs, crop, psi correction     */
  LAMINO_STAGE_X3 = 3,       /* transform along x3                          */
  LAMINO_NSTAGE = 4
};

/* Turn per-stage timing of later calls on (enable != 0) or off.  When on,
 * every call records HIP events on its own stream around each stage's
 * kernels (a small overhead per launch).  Host-only. */
int lamino_plan_profile(lamino_plan_t* plan, int enable);

/* Accumulated device milliseconds and kernel-launch counts per stage over
 * the calls made while timing was on; ms and launches are arrays of
 * LAMINO_NSTAGE entries (either may be NULL).  Waits for the recorded
 * events.  reset != 0 clears the accumulators afterwards.  Errors:
 * E_INVALID, E_HIP. */
int lamino_plan_stage_times(lamino_plan_t* plan, double* ms, int* launches, int reset);

/* ---------------------------------------------------------------------
 * Total-variation regularised reconstruction (Appendix A).
 *
 * The problem is min 1/2 ||L mu - d||^2 + alpha sum_v |grad mu (v)|
 * (eq:mainregproblem, isotropic TV).  Discrete operators on a float32
 * volume vol[nz][ny][nx] (x fastest):
 *   grad: forward differences, g[c][z][y][x] with c = 0 (x), 1 (y), 2 (z);
 *         the last difference along each axis is 0;
 *   div:  -grad^T (the paper defines div as the adjoint of -grad).
 * Gradient fields are component-major float32 arrays [3][nz][ny][nx].
 * Input and output buffers of one call must not overlap unless stated.
 * These calls need no plan; sizes must be positive (E_INVALID) and the
 * volume at most 2^30 tiles of 64 x 4 x 16 voxels (E_UNSUPPORTED). */

/* d_grad = grad d_vol. */
int lamino_tv_grad(const float* d_vol, float* d_grad, int nz, int ny, int nx, void* stream);

/* d_out = div d_p = -grad^T d_p. */
int lamino_tv_div(const float* d_p, float* d_out, int nz, int ny, int nx, void* stream);

/* d_out = d_base - rho div(grad d_vol - d_shift): the gradient of
 * rho/2 ||grad vol - shift||^2 added to base, i.e. the regularisation part
 * of the sub-problem gradient Eq:gradtomo with shift = psi - lambda / rho.
 * d_shift and d_base may be NULL (zero).  d_out may equal d_base. */
int lamino_tv_term(const float* d_vol, const float* d_shift, const float* d_base, double rho,
                   float* d_out, int nz, int ny, int nx, void* stream);

/* The psi-step and dual update of the ADMM (Eq:reg, Eq:lamd), per voxel on
 * the 3-vectors g = grad vol (v):
 *   psi = shrink(g + lambda / rho, alpha / rho),
 *         shrink(q, t) = q max(0, 1 - t / |q|)   (the minimiser of the
 *         augmented Lagrangian eq:alagr as written: thresholds lambda/rho
 *         and alpha/rho),
 *   lambda <- lambda + rho (g - psi)              (d_lambda updated in place),
 *   d_shift = psi - lambda / rho (new lambda)     (what the next sub-problem
 *                                                  needs),
 *   d_psi = psi if d_psi != NULL.
 * Needs rho > 0, alpha >= 0 (E_INVALID). */
int lamino_tv_shrink(const float* d_vol, float* d_lambda, float* d_shift, float* d_psi,
                     double alpha, double rho, int nz, int ny, int nx, void* stream);

/* Bytes of the device state buffer lamino_admm_tv needs for this plan's
 * volume and detector (about 10 volumes plus one data array).  Host-only. */
int lamino_admm_tv_state_bytes(const lamino_plan_t* plan, size_t* bytes);

/* ADMM for eq:mainregproblem with this plan's L and L* (Appendix A).
 * outer iterations, each:
 *   mu <- `inner` conjugate-gradient steps on Eq:tomo from the current mu
 *         (gradient Eq:gradtomo, Dai-Yuan direction Eq:DaiYuan2, exact line
 *         search gamma = -<g, eta> / (||L eta||^2 + rho ||grad eta||^2),
 *         restarted from the steepest-descent direction each iteration);
 *   psi, lambda <- lamino_tv_shrink.
 * A zero line-search or Dai-Yuan denominator ends that inner solve early.
 * d_data: float32 d[n_theta][h][w] (the plan's data dtype must be F32,
 * E_INVALID otherwise; the storage dtype may be narrower).  d_vol: the
 * initial guess on entry, the result on exit.  d_state: caller-owned
 * device buffer of lamino_admm_tv_state_bytes bytes, 256-byte aligned,
 * laid out as lambda [3][nz][n][n] float32 at offset 0, then (at the next
 * 256-byte boundary) shift = psi - lambda / rho [3][nz][n][n] float32,
 * then work arrays.  resume == 0 starts from psi = lambda = 0 and forms
 * L*(L mu - d) from d_vol (one L and one L*); resume != 0 continues from a
 * previous call's state with the same plan, data, volume buffer and rho.
 * Cost per outer iteration: `inner` (L + L*) plus bandwidth-bound volume
 * kernels; every scalar stays on the device (no host synchronisation).
 * Errors: E_INVALID, E_UNBOUND, E_UNSUPPORTED, E_HIP. */
int lamino_admm_tv(const lamino_plan_t* plan, const float* d_data, float* d_vol, double alpha,
                   double rho, int outer, int inner, int resume, void* d_state, void* stream);

/* ---------------------------------------------------------------------
 * Allocation-free filtered backprojection, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same operation and arguments as
 * lamino_fbp, but the plan's tables and workspace live in a device array of
 * LAMINO_SCRATCH_BYTES bytes inside the library (one per device, held from
 * the first call on that device until the process ends) instead of
 * caller-bound buffers: the plan need not be bound, and nothing is
 * allocated.  The caller passes the device input d[n_theta][h][w] and the
 * output vol[nz][n][n] as for lamino_fbp.  Each call uploads the plan's
 * table image into the array on `stream` (the plan must outlive the call's
 * completion).  All calls on one device share the array: calls that overlap
 * on a device race (serialise them on one stream).  Stage timing
 * (lamino_plan_profile) does not apply.  Errors: E_INVALID (NULL
 * arguments), E_BUDGET (table + workspace bytes above LAMINO_SCRATCH_BYTES;
 * a plan made with opts.hbm_budget well below the limit fits), E_HIP. */
#define LAMINO_SCRATCH_BYTES (64u << 20)
int lamino_fbp_noalloc(const lamino_plan_t* plan, const void* d_data, float* d_vol, void* stream);

/* Free the host plan (device buffers stay with the caller). NULL is ok. */
int lamino_plan_destroy(lamino_plan_t* plan);

/* Static description of a status code. */
const char* lamino_strerror(int status);

/* Thread-local message of the last failure on this thread ("" if none). */
const char* lamino_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LAMINO_H */
