// Internal plan layout and kernel launch interface.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/lamino.h"

namespace lam {

// Parameters every kernel receives by value (device pointers into the
// caller's table and workspace buffers).
struct KParams {
  int nz, n, n_theta, h, w;
  int h_p, w_p, n_slab, grid, M;
  int log2_hp, log2_wp, log2_grid, log2_twmax;
  float beta;
  float ncw;       // grid / w_p
  float gs;        // grid * sin(phi) / h_p (per unit of l)
  int data_dtype, storage_dtype;
  const float2* trig;     // [n_theta] (cos, sin)
  const float* filt;      // [w_p] transfer function incl. 1/(h_p w_p)
  const float* deapod;    // [n] psi correction per axis
  // x3 transform operands (matrix-core layout, 16-bit hi and lo planes):
  //   adj: A[z][2l + c] = w_l (cos a, -sin a)[c], a = 2 pi x3 l cos(phi) / h_p,
  //        rows padded to x3a_rows, K = x3a_k; bf16 (f16 for float16 storage)
  //   fwd: A[2l + c][z] = (cos a, -sin a)[c], rows x3f_rows, K = x3f_k; bf16
  //   fragment-major: (row, k) at ((k / 16 * rows + row) * 2 + k % 16 / 8) * 8 + k % 8
  const unsigned short* x3a;  // [2][x3a_rows][x3a_k]
  const unsigned short* x3f;  // [2][x3f_rows][x3f_k]
  int x3a_rows, x3a_k, x3f_rows, x3f_k;
  float x3_out_scale;     // 1 / (power-of-two factor carried by the stored spectra)
  // float16 range control of the forward direction (1 for other storage):
  // exact powers of two carried by the stored slab planes g and spectra D
  float fwd_g_scale, fwd_D_scale;
  // float16 storage: device [f, 1/f], f = 2^-e with the call's input scaled
  // into [0.5, 1) by f (first kernel) and the output by 1/f (last kernel);
  // NULL for other storage types
  const float* dyn;
  const float2* tw;       // [2^log2_twmax] exp(-2 pi i t / 2^log2_twmax)
  // direct (line-integral) path
  const double2* trig_d;  // [n_theta] (cos, sin) in double precision
  const float* filt_dir;  // [w_p] W(m) / w_p of the row filter, index k = m mod w_p
  double sin_phi, cos_phi;
  // raw-count prologue of the first detector kernel (dark == NULL: none)
  const float* dark;      // [h][w]
  const float* flat;      // [h][w]
  float min_ratio;
};

}  // namespace lam

struct lamino_plan_s {
  // geometry
  int nz, n, n_theta, h, w;
  double tilt;
  std::vector<double> theta;
  lamino_opts opts;
  // derived sizes
  int h_p, w_p, n_slab, grid, M, tile;
  double beta;
  int z_chunk, slab_chunk, theta_chunk;
  // table layout (bytes)
  size_t off_trig, off_filt_fbp, off_filt_adj, off_deapod, off_x3a, off_x3f, off_tw;
  size_t off_trig_d, off_filt_dir;
  double spectra_scale;  // power of two folded into the FBP filter table
  double adj_scale;      // the same for the L* filter table
  int x3a_rows, x3a_k, x3f_rows, x3f_k;
  size_t table_bytes;
  int log2_twmax;
  // workspace layout (bytes)
  size_t off_w1, off_D, off_G, off_g, off_phase, off_dyn;
  size_t bytes_w1, bytes_D, bytes_G, bytes_g;
  size_t work_bytes;
  // Out-of-core layout: when the resident workspace exceeds opts.hbm_budget
  // the spectra D and / or the slab planes g live in a caller-owned host
  // buffer (host_bytes; D at off_hD, g at off_hg) and the device workspace
  // holds double-buffered chunks instead: D[l][theta chunk][k] written by the
  // detector stage (off_Dout), D[slab chunk][theta][k] read by gridding
  // (off_Din), g[slab chunk][y][x] written by the slab stage (off_gout) and
  // g[l][column chunk] read by the x3 transform (off_gcol, col_chunk columns).
  bool spill_D, spill_g;
  int col_chunk;
  size_t off_Dout[2], off_Din[2], off_gout[2], off_gcol[2];
  size_t host_bytes, off_hD, off_hg;
  void* h_spill;
  // host-memory input / output (lamino_fbp_host): device staging buffer of
  // io_bytes with data chunks [theta_chunk][h][w] at off_in[] and volume
  // chunks at off_vout[] (io_z slices, or all slices of col_chunk columns
  // when g is spilled)
  int io_z;
  size_t off_in[2], off_vout[2], io_bytes;
  // streams and events of the out-of-core pipeline (created on first use)
  hipStream_t s_in, s_out;
  hipEvent_t ev[16];
  bool pipe_ready;
  std::vector<unsigned char> host_tables;
  void* d_tables;
  void* d_work;
  bool bound;
  // per-stage timing: event pairs recorded on the call's stream
  bool profiling;
  struct Mark {
    int stage;
    int launches;
    hipEvent_t start, stop;
  };
  std::vector<Mark> marks;            // recorded, not yet collected
  std::vector<hipEvent_t> event_pool; // created events available for reuse
  double stage_ms[LAMINO_NSTAGE];
  int stage_launches[LAMINO_NSTAGE];
};

namespace lam {

// Kernel parameters with the table and workspace pointers of the plan's
// bound buffers, or of the buffers given (tables / work not NULL).
KParams make_params(const lamino_plan_s* p, bool fbp_filter, const void* tables = nullptr,
                    void* work = nullptr);
// Records a thread-local error message (lamino_last_error) and returns code.
int api_fail(int code, const char* fmt, ...);
size_t storage_bytes(int dtype);  // bytes of one stored complex value
size_t data_bytes(int dtype);     // bytes of one real data value
bool integer_dtype(int dtype);    // U8 / U16: input-only data types

// Stage bracketing (no-ops unless profiling is on).
struct StageTimer {
  lamino_plan_s* p;
  hipStream_t s;
  int stage, launches;
  hipEvent_t start;
  StageTimer(const lamino_plan_s* plan, hipStream_t stream, int stage_id, int nlaunch,
             bool enabled = true);
  ~StageTimer();
};

// The three operator pipelines (enqueue only).
// Optional parts of a backprojection: the raw-count prologue (dark != NULL),
// a rotation-axis offset (detector columns; applied as a phase ramp on the
// row spectra) and the output slices [z_first, z_first + z_count) written
// to d_vol[0 .. z_count).
// Device buffers other than the plan's bound ones (tables / work not NULL,
// same layouts), and stage timing off (timing = false: no events created).
struct BackprojOpts {
  const float* dark = nullptr;
  const float* flat = nullptr;
  float min_ratio = 0.f;
  double center_shift = 0.0;
  int z_first = 0;
  int z_count = -1;  // -1: all nz slices
  const void* tables = nullptr;
  void* work = nullptr;
  bool timing = true;
  // host-memory input and output streamed through the staging buffer io
  // (lamino_fbp_host); d_data / d_vol are then NULL
  const void* h_data = nullptr;
  float* h_vol = nullptr;
  void* io = nullptr;
};
hipError_t run_backprojection(const lamino_plan_s* p, const void* d_data, float* d_vol,
                              bool fbp_filter, hipStream_t s, const BackprojOpts& o = BackprojOpts());
// Creates the pipeline streams and events of a plan (no-op after the first call).
hipError_t ensure_pipe(lamino_plan_s* p);
hipError_t run_forward(const lamino_plan_s* p, const float* d_vol, void* d_data,
                       hipStream_t s);

// Direct line-integral backprojection (enqueue only); d_work holds the
// filtered rows when fbp_filter is set.
size_t direct_work_bytes(const lamino_plan_s* p);
hipError_t run_direct(const lamino_plan_s* p, const void* d_data, float* d_vol, void* d_work,
                      bool fbp_filter, hipStream_t s);

// Total-variation operators and the ADMM driver (enqueue only).
size_t admm_state_bytes(const lamino_plan_s* p);
bool tv_dims_ok(int nz, int ny, int nx);
hipError_t tv_grad(const float* mu, float* out, int nz, int ny, int nx, hipStream_t s);
hipError_t tv_div(const float* p, float* out, int nz, int ny, int nx, hipStream_t s);
hipError_t tv_term(const float* mu, const float* shift, const float* base, float rho, float* out,
                   int nz, int ny, int nx, hipStream_t s);
hipError_t tv_shrink(const float* mu, float* lam, float* shift, float* psi, float alpha, float rho,
                     int nz, int ny, int nx, hipStream_t s);
hipError_t run_admm_tv(const lamino_plan_s* p, const float* d_data, float* mu, float alpha,
                       float rho, int outer, int inner, int resume, void* state, hipStream_t s);

}  // namespace lam
