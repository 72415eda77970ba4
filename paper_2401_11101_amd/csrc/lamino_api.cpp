// Host side of the C ABI: validation, double-precision tables, workspace
// layout, binding and the three operator entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "lamino_common.h"
#include "lamino_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_fail(hipError_t e, const char* where) {
  return fail(LAMINO_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

int pow2_at_least(double x) {
  long p = 1;
  while ((double)p < x && p < (1L << 30)) p *= 2;
  return (int)p;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Transfer-function windows of the FBP filter, k in cycles per pixel.
double window(double k, int kind) {
  k = std::fabs(k);
  if (kind == LAMINO_RAMP) return 1.0;
  if (kind == LAMINO_SHEPP_LOGAN) return k == 0.0 ? 1.0 : std::sin(M_PI * k) / (M_PI * k);
  const double t = 2.0 * k;  // Parzen on [-1/2, 1/2]
  if (t <= 0.5) return 1.0 - 6.0 * t * t * (1.0 - t);
  if (t <= 1.0) return 2.0 * (1.0 - t) * (1.0 - t) * (1.0 - t);
  return 0.0;
}

constexpr size_t kChunkTarget = 512u << 20;  // bytes per chunked intermediate
constexpr int kAbsmaxBlocks = 1024;          // partial maxima of the float16 input scan

void layout_work(lamino_plan_s* p) {
  const size_t sb = lam::storage_bytes(p->opts.storage_dtype);
  const size_t ncol = (size_t)p->n * p->n;
  p->bytes_w1 = (size_t)p->theta_chunk * p->n_slab * p->w * 8;
  p->bytes_D = (size_t)p->n_slab * p->n_theta * p->w_p * sb;
  p->bytes_G = (size_t)p->slab_chunk * p->grid * p->grid * 8;
  p->bytes_g = (size_t)p->n_slab * ncol * sb;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  p->off_w1 = take(p->bytes_w1);
  p->off_D = 0;
  if (!p->spill_D) {
    p->off_D = take(p->bytes_D);
  } else {
    for (int i = 0; i < 2; ++i) p->off_Dout[i] = take((size_t)p->n_slab * p->theta_chunk * p->w_p * sb);
    for (int i = 0; i < 2; ++i) p->off_Din[i] = take((size_t)p->slab_chunk * p->n_theta * p->w_p * sb);
  }
  p->off_G = take(p->bytes_G);
  p->off_g = 0;
  if (!p->spill_g) {
    p->off_g = take(p->bytes_g);
  } else {
    for (int i = 0; i < 2; ++i) p->off_gout[i] = take((size_t)p->slab_chunk * ncol * sb);
    for (int i = 0; i < 2; ++i) p->off_gcol[i] = take((size_t)p->n_slab * p->col_chunk * sb);
  }
  p->off_phase = take((size_t)p->w_p * 8);  // rotation-axis phase ramp, w_p complex values
  // float16 per-call input factor and block partial maxima
  p->off_dyn = take((size_t)(2 + kAbsmaxBlocks) * 4);
  p->work_bytes = off;
  // host spill buffer
  size_t h = 0;
  p->off_hD = p->off_hg = 0;
  if (p->spill_D) {
    p->off_hD = h;
    h += align256(p->bytes_D);
  }
  if (p->spill_g) {
    p->off_hg = h;
    h += align256(p->bytes_g);
  }
  p->host_bytes = h;
  // staging buffer of lamino_fbp_host
  size_t io = 0;
  for (int i = 0; i < 2; ++i) {
    p->off_in[i] = io;
    io += align256((size_t)p->theta_chunk * p->h * p->w * lam::data_bytes(p->opts.data_dtype));
  }
  for (int i = 0; i < 2; ++i) {
    p->off_vout[i] = io;
    io += align256(p->spill_g ? (size_t)p->nz * p->col_chunk * 4 : (size_t)p->io_z * ncol * 4);
  }
  p->io_bytes = io;
}

// Halve the chunk whose buffers take the most workspace until the layout fits
// `budget` or every chunk is down to one unit; returns whether it fits.
bool shrink_to_budget(lamino_plan_s* p, size_t budget) {
  const size_t sb = lam::storage_bytes(p->opts.storage_dtype);
  const size_t ncol = (size_t)p->n * p->n;
  layout_work(p);
  while (p->work_bytes > budget) {
    const size_t by_theta = p->bytes_w1 + (p->spill_D ? 2 * (size_t)p->n_slab * p->theta_chunk * p->w_p * sb : 0);
    const size_t by_slab = p->bytes_G + (p->spill_D ? 2 * (size_t)p->slab_chunk * p->n_theta * p->w_p * sb : 0) +
                           (p->spill_g ? 2 * (size_t)p->slab_chunk * ncol * sb : 0);
    const size_t by_col = p->spill_g ? 2 * (size_t)p->n_slab * p->col_chunk * sb : 0;
    if (p->slab_chunk > 1 && by_slab >= by_theta && by_slab >= by_col) {
      p->slab_chunk = (p->slab_chunk + 1) / 2;
    } else if (p->theta_chunk > 1 && by_theta >= by_col) {
      p->theta_chunk = (p->theta_chunk + 1) / 2;
    } else if (p->spill_g && p->col_chunk > 256) {
      p->col_chunk = std::max(256, p->col_chunk / 2 / 256 * 256);
    } else if (p->slab_chunk > 1) {
      p->slab_chunk = (p->slab_chunk + 1) / 2;
    } else if (p->theta_chunk > 1) {
      p->theta_chunk = (p->theta_chunk + 1) / 2;
    } else {
      return false;
    }
    layout_work(p);
  }
  return true;
}

int round_up(int a, int b) { return (a + b - 1) / b * b; }

// Round-to-nearest-even bfloat16 / float16 bits of x.
unsigned short to_bf16(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
float from_bf16(unsigned short h) {
  const uint32_t u = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &u, 4);
  return x;
}
// x ~ hi + lo with hi, lo 16-bit floats (bfloat16, or float16 if f16)
void split16(double x, bool f16, unsigned short& hi, unsigned short& lo) {
  if (f16) {
    const _Float16 h = (_Float16)x;
    const _Float16 l = (_Float16)(x - (double)h);
    std::memcpy(&hi, &h, 2);
    std::memcpy(&lo, &l, 2);
  } else {
    hi = to_bf16((float)x);
    lo = to_bf16((float)(x - (double)from_bf16(hi)));
  }
}

void build_tables(lamino_plan_s* p) {
  const double phi = p->tilt;
  const double cphi = std::cos(phi);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(bytes);
    return o;
  };
  const int twmax = std::max(std::max(p->h_p, p->w_p), p->grid);
  p->log2_twmax = lam::ilog2(twmax);
  p->off_trig = take((size_t)p->n_theta * 8);
  p->off_filt_fbp = take((size_t)p->w_p * 4);
  p->off_filt_adj = take((size_t)p->w_p * 4);
  p->off_deapod = take((size_t)p->n * 4);
  p->x3a_rows = round_up(p->nz, 32);
  p->x3a_k = round_up(2 * p->n_slab, 16);
  p->x3f_rows = round_up(2 * p->n_slab, 32);
  p->x3f_k = round_up(p->nz, 16);
  p->off_x3a = take((size_t)2 * p->x3a_rows * p->x3a_k * 2);
  p->off_x3f = take((size_t)2 * p->x3f_rows * p->x3f_k * 2);
  p->off_tw = take((size_t)twmax * 8);
  p->off_trig_d = take((size_t)p->n_theta * 16);
  p->off_filt_dir = take((size_t)p->w_p * 4);
  p->table_bytes = off;
  p->host_tables.assign(off, 0);
  unsigned char* base = p->host_tables.data();

  float* trig = reinterpret_cast<float*>(base + p->off_trig);
  for (int j = 0; j < p->n_theta; ++j) {
    trig[2 * j] = (float)std::cos(p->theta[j]);
    trig[2 * j + 1] = (float)std::sin(p->theta[j]);
  }
  // W(m) / (h_p w_p) for FBP and 1 / (h_p w_p) for L*, indexed by k = m mod w_p;
  // the Nyquist bin k = w_p / 2 is not part of the sums.
  float* ffbp = reinterpret_cast<float*>(base + p->off_filt_fbp);
  float* fadj = reinterpret_cast<float*>(base + p->off_filt_adj);
  // Float16 storage: the filtered spectra carry an extra power-of-two factor
  // s = h_p w_p / 64 (exact), which keeps their typical magnitudes away from
  // the float16 subnormal range; the x3 transform multiplies its output by 1/s.
  p->spectra_scale = p->opts.storage_dtype == LAMINO_F16 ? (double)p->h_p * p->w_p / 64.0 : 1.0;
  // L* lacks the filter's pi / n_theta: its spectra and slab planes are
  // ~n_theta times larger, so its factor is smaller by the next power of two
  p->adj_scale = p->opts.storage_dtype == LAMINO_F16 ? p->spectra_scale / pow2_at_least(p->n_theta)
                                                      : 1.0;
  const double norm = p->spectra_scale / ((double)p->h_p * p->w_p);
  const double norm_adj = p->adj_scale / ((double)p->h_p * p->w_p);
  for (int k = 0; k < p->w_p; ++k) {
    const int m = k < p->w_p / 2 ? k : k - p->w_p;
    const double km = (double)m / p->w_p;
    const bool nyq = (k == p->w_p / 2);
    ffbp[k] = nyq ? 0.f
                  : (float)(M_PI / p->n_theta * cphi * std::fabs(km) * window(km, p->opts.filter) * norm);
    fadj[k] = nyq ? 0.f : (float)norm_adj;
  }
  // psi correction of the Gaussian USFFT per axis
  float* deap = reinterpret_cast<float*>(base + p->off_deapod);
  for (int i = 0; i < p->n; ++i) {
    const double x = i - p->n / 2;
    deap[i] = (float)(std::sqrt(p->beta / M_PI) *
                      std::exp(M_PI * M_PI * x * x / (p->beta * (double)p->grid * p->grid)));
  }
  // x3 phases: xi3 = l cos(phi) / h_p (eq:uneqspace), as hi + lo pairs of
  // 16-bit values for the matrix-core x3 transforms.  Fragment-major layout:
  // entry (row, k) sits at ((k / 16 * rows + row) * 2 + k % 16 / 8) * 8 + k % 8,
  // so the 8-value operand of every lane of a 32-row tile is one contiguous run.
  unsigned short* xa = reinterpret_cast<unsigned short*>(base + p->off_x3a);
  unsigned short* xf = reinterpret_cast<unsigned short*>(base + p->off_x3f);
  const size_t pa = (size_t)p->x3a_rows * p->x3a_k, pf = (size_t)p->x3f_rows * p->x3f_k;
  auto frag = [](size_t rows, size_t row, size_t k) {
    return ((k / 16 * rows + row) * 2 + (k % 16) / 8) * 8 + k % 8;
  };
  const bool f16a = p->opts.storage_dtype == LAMINO_F16;
  for (int z = 0; z < p->nz; ++z) {
    const double x3 = z - p->nz / 2;
    for (int l = 0; l < p->n_slab; ++l) {
      const double a = 2.0 * M_PI * x3 * l * cphi / p->h_p;
      const double wl = l == 0 ? 1.0 : 2.0;
      const double va[2] = {wl * std::cos(a), -wl * std::sin(a)};
      const double vf[2] = {std::cos(a), -std::sin(a)};
      for (int c = 0; c < 2; ++c) {
        const size_t ia = frag(p->x3a_rows, z, 2 * l + c);
        split16(va[c], f16a, xa[ia], xa[pa + ia]);
        const size_t jf = frag(p->x3f_rows, 2 * l + c, z);
        split16(vf[c], false, xf[jf], xf[pf + jf]);
      }
    }
  }
  float* tw = reinterpret_cast<float*>(base + p->off_tw);
  for (int t = 0; t < twmax; ++t) {
    const double a = -2.0 * M_PI * t / twmax;
    tw[2 * t] = (float)std::cos(a);
    tw[2 * t + 1] = (float)std::sin(a);
  }
  // direct path: angles in double precision, row filter W(m) / w_p
  double* trd = reinterpret_cast<double*>(base + p->off_trig_d);
  for (int j = 0; j < p->n_theta; ++j) {
    trd[2 * j] = std::cos(p->theta[j]);
    trd[2 * j + 1] = std::sin(p->theta[j]);
  }
  float* fdir = reinterpret_cast<float*>(base + p->off_filt_dir);
  for (int k = 0; k < p->w_p; ++k) {
    const int m = k < p->w_p / 2 ? k : k - p->w_p;
    const double km = (double)m / p->w_p;
    fdir[k] = k == p->w_p / 2 ? 0.f
                              : (float)(M_PI / p->n_theta * cphi * std::fabs(km) *
                                        window(km, p->opts.filter) / p->w_p);
  }
}

}  // namespace

namespace lam {

int api_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

size_t storage_bytes(int dtype) { return dtype == LAMINO_F32 ? 8 : 4; }
size_t data_bytes(int dtype) { return dtype == LAMINO_F32 ? 4 : (dtype == LAMINO_U8 ? 1 : 2); }
bool integer_dtype(int dtype) { return dtype == LAMINO_U8 || dtype == LAMINO_U16; }

KParams make_params(const lamino_plan_s* p, bool fbp_filter, const void* tables, void* work) {
  if (!tables) tables = p->d_tables;
  if (!work) work = p->d_work;
  KParams k;
  k.nz = p->nz;
  k.n = p->n;
  k.n_theta = p->n_theta;
  k.h = p->h;
  k.w = p->w;
  k.h_p = p->h_p;
  k.w_p = p->w_p;
  k.n_slab = p->n_slab;
  k.grid = p->grid;
  k.M = p->M;
  k.log2_hp = ilog2(p->h_p);
  k.log2_wp = ilog2(p->w_p);
  k.log2_grid = ilog2(p->grid);
  k.log2_twmax = p->log2_twmax;
  k.beta = (float)p->beta;
  k.ncw = (float)((double)p->grid / p->w_p);
  k.gs = (float)((double)p->grid * std::sin(p->tilt) / p->h_p);
  k.data_dtype = p->opts.data_dtype;
  k.storage_dtype = p->opts.storage_dtype;
  const char* t = static_cast<const char*>(tables);
  k.trig = reinterpret_cast<const float2*>(t + p->off_trig);
  k.filt = reinterpret_cast<const float*>(t + (fbp_filter ? p->off_filt_fbp : p->off_filt_adj));
  k.deapod = reinterpret_cast<const float*>(t + p->off_deapod);
  k.x3a = reinterpret_cast<const unsigned short*>(t + p->off_x3a);
  k.x3f = reinterpret_cast<const unsigned short*>(t + p->off_x3f);
  k.x3_out_scale = (float)(1.0 / (fbp_filter ? p->spectra_scale : p->adj_scale));
  if (p->opts.storage_dtype == LAMINO_F16) {
    // forward direction, input scaled into [0.5, 1): the slab planes sum nz
    // voxels (factor 1 / 2^ceil(log2 nz)); the spectra sum the (1.45 n)^2
    // psi-corrected plane values times at most ~13 Gaussian tap weights,
    // kept below 2^15 by 2^15 / 2^ceil(log2(32 n^2))
    k.fwd_g_scale = (float)(1.0 / pow2_at_least(p->nz));
    k.fwd_D_scale = (float)(32768.0 / pow2_at_least(32.0 * p->n * p->n));
    k.dyn = reinterpret_cast<const float*>(static_cast<const char*>(work) + p->off_dyn);
  } else {
    k.fwd_g_scale = 1.f;
    k.fwd_D_scale = 1.f;
    k.dyn = nullptr;
  }
  k.x3a_rows = p->x3a_rows;
  k.x3a_k = p->x3a_k;
  k.x3f_rows = p->x3f_rows;
  k.x3f_k = p->x3f_k;
  k.tw = reinterpret_cast<const float2*>(t + p->off_tw);
  k.trig_d = reinterpret_cast<const double2*>(t + p->off_trig_d);
  k.filt_dir = reinterpret_cast<const float*>(t + p->off_filt_dir);
  k.sin_phi = std::sin(p->tilt);
  k.cos_phi = std::cos(p->tilt);
  k.dark = nullptr;
  k.flat = nullptr;
  k.min_ratio = 0.f;
  return k;
}

hipError_t ensure_pipe(lamino_plan_s* p) {
  if (p->pipe_ready) return hipSuccess;
  hipError_t e = hipStreamCreateWithFlags(&p->s_in, hipStreamNonBlocking);  // default priority
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&p->s_out, hipStreamNonBlocking);
  for (auto& ev : p->ev)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
  if (e == hipSuccess) p->pipe_ready = true;
  return e;
}

static hipEvent_t take_event(lamino_plan_s* p) {
  if (!p->event_pool.empty()) {
    hipEvent_t e = p->event_pool.back();
    p->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

StageTimer::StageTimer(const lamino_plan_s* plan, hipStream_t stream, int stage_id, int nlaunch,
                       bool enabled)
    : p(const_cast<lamino_plan_s*>(plan)), s(stream), stage(stage_id), launches(nlaunch),
      start(nullptr) {
  if (!p->profiling || !enabled) return;
  start = take_event(p);
  if (start) (void)hipEventRecord(start, s);
}

StageTimer::~StageTimer() {
  if (!start) return;
  hipEvent_t stop = take_event(p);
  if (!stop) return;
  (void)hipEventRecord(stop, s);
  p->marks.push_back({stage, launches, start, stop});
}

}  // namespace lam

extern "C" {

int lamino_plan_profile(lamino_plan_t* p, int enable) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_profile: NULL plan");
  p->profiling = enable != 0;
  return LAMINO_OK;
}

int lamino_plan_stage_times(lamino_plan_t* p, double* ms, int* launches, int reset) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_stage_times: NULL plan");
  for (auto& m : p->marks) {
    hipError_t e = hipEventSynchronize(m.stop);
    if (e != hipSuccess) return hip_fail(e, "lamino_plan_stage_times");
    float t = 0.f;
    e = hipEventElapsedTime(&t, m.start, m.stop);
    if (e != hipSuccess) return hip_fail(e, "lamino_plan_stage_times");
    p->stage_ms[m.stage] += t;
    p->stage_launches[m.stage] += m.launches;
    p->event_pool.push_back(m.start);
    p->event_pool.push_back(m.stop);
  }
  p->marks.clear();
  for (int i = 0; i < LAMINO_NSTAGE; ++i) {
    if (ms) ms[i] = p->stage_ms[i];
    if (launches) launches[i] = p->stage_launches[i];
    if (reset) {
      p->stage_ms[i] = 0.0;
      p->stage_launches[i] = 0;
    }
  }
  return LAMINO_OK;
}


void lamino_opts_default(lamino_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->data_dtype = LAMINO_F32;
  o->storage_dtype = LAMINO_F32;
  o->filter = LAMINO_SHEPP_LOGAN;
  o->pad_u = 2.0;
  o->pad_v = 2.0;
}

int lamino_plan(const lamino_geom* geom, const lamino_opts* opts, lamino_plan_t** out) {
  g_last_error.clear();
  if (!geom || !out) return fail(LAMINO_E_INVALID, "lamino_plan: NULL geometry or output");
  *out = nullptr;
  lamino_opts o;
  lamino_opts_default(&o);
  if (opts) o = *opts;
  if (geom->nz < 1 || geom->n < 1 || geom->n_theta < 1 || geom->h < 1 || geom->w < 1)
    return fail(LAMINO_E_INVALID, "lamino_plan: sizes must be positive (nz=%d n=%d n_theta=%d h=%d w=%d)",
                geom->nz, geom->n, geom->n_theta, geom->h, geom->w);
  if (geom->n_theta > 65535)
    return fail(LAMINO_E_UNSUPPORTED, "lamino_plan: n_theta=%d above 65535", geom->n_theta);
  if (!std::isfinite(geom->tilt) || std::fabs(geom->tilt) >= M_PI / 2)
    return fail(LAMINO_E_INVALID, "lamino_plan: tilt must be finite with |tilt| < pi/2");
  if (o.data_dtype < 0 || o.data_dtype > 4 || o.storage_dtype < 0 || o.storage_dtype > 2)
    return fail(LAMINO_E_INVALID, "lamino_plan: unknown dtype");
  if (o.filter < 0 || o.filter > 2) return fail(LAMINO_E_INVALID, "lamino_plan: unknown filter");
  if (o.pad_u == 0.0) o.pad_u = 2.0;
  if (o.pad_v == 0.0) o.pad_v = 2.0;
  if (!(o.pad_u >= 1.0) || !(o.pad_v >= 1.0) || !std::isfinite(o.pad_u) || !std::isfinite(o.pad_v))
    return fail(LAMINO_E_INVALID, "lamino_plan: padding factors must be >= 1");
  if (o.kernel_m != 0 && (o.kernel_m < 2 || o.kernel_m > 8))
    return fail(LAMINO_E_INVALID, "lamino_plan: kernel_m must be 0 or 2..8");
  if (o.z_chunk < 0 || o.slab_chunk < 0 || o.theta_chunk < 0)
    return fail(LAMINO_E_INVALID, "lamino_plan: chunk sizes must be >= 0");

  lamino_plan_s* p = new (std::nothrow) lamino_plan_s();
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan: out of host memory");
  p->nz = geom->nz;
  p->n = geom->n;
  p->n_theta = geom->n_theta;
  p->h = geom->h;
  p->w = geom->w;
  p->tilt = geom->tilt;
  p->opts = o;
  p->theta.resize(p->n_theta);
  for (int j = 0; j < p->n_theta; ++j) {
    p->theta[j] = geom->theta ? geom->theta[j] : 2.0 * M_PI * j / p->n_theta;
    if (!std::isfinite(p->theta[j])) {
      delete p;
      return fail(LAMINO_E_INVALID, "lamino_plan: theta[%d] is not finite", j);
    }
  }
  p->w_p = pow2_at_least(std::ceil(o.pad_u * p->w));
  p->h_p = pow2_at_least(std::ceil(o.pad_v * p->h));
  // the gridding works on 32 x 32 matrix-core tiles
  p->grid = std::max(32, pow2_at_least(2.0 * p->n));
  if (p->w_p < 2 || p->h_p < 2 || p->w_p > 8192 || p->h_p > 8192 || p->grid > 8192) {
    const int wp = p->w_p, hp = p->h_p, gr = p->grid;
    delete p;
    return fail(LAMINO_E_UNSUPPORTED,
                "lamino_plan: FFT sizes w_p=%d h_p=%d grid=%d outside [2, 8192]", wp, hp, gr);
  }
  p->n_slab = p->h_p / 2;
  p->M = o.kernel_m ? o.kernel_m : (o.storage_dtype == LAMINO_F32 ? 5 : 3);
  {
    // Gaussian width of Greengard & Lee (2004) for oversampling R = grid / n,
    // expressed in grid cells: phi(t) = exp(-beta t^2).
    const double R = (double)p->grid / p->n;
    p->beta = M_PI * (R - 0.5) / (R * p->M);
  }
  p->tile = 0;
  p->z_chunk = o.z_chunk ? std::min(o.z_chunk, p->nz) : p->nz;
  const size_t ncol = (size_t)p->n * p->n;
  const size_t slab_bytes = (size_t)p->grid * p->grid * 8;
  const size_t w1_bytes = (size_t)p->n_slab * p->w * 8;
  const int slab_auto = (int)std::max<size_t>(1, std::min<size_t>(p->n_slab, kChunkTarget / slab_bytes));
  const int theta_auto = (int)std::max<size_t>(1, std::min<size_t>(p->n_theta, kChunkTarget / w1_bytes));
  // host-output slices per chunk and x3 columns per chunk of spilled slab planes
  p->io_z = o.z_chunk ? p->z_chunk
                      : (int)std::max<size_t>(1, std::min<size_t>(p->nz, kChunkTarget / (ncol * 4)));
  const size_t sb = lam::storage_bytes(o.storage_dtype);
  const int col_auto = (int)std::max<size_t>(
      256, std::min<size_t>((ncol + 255) / 256 * 256, kChunkTarget / (p->n_slab * sb) / 256 * 256));
  p->spill_D = p->spill_g = false;
  p->h_spill = nullptr;
  p->s_in = p->s_out = nullptr;
  p->pipe_ready = false;
  for (auto& e : p->ev) e = nullptr;
  auto reset_chunks = [&]() {
    p->slab_chunk = o.slab_chunk ? std::min(o.slab_chunk, p->n_slab) : slab_auto;
    p->theta_chunk = o.theta_chunk ? std::min(o.theta_chunk, p->n_theta) : theta_auto;
    p->col_chunk = col_auto;
  };
  reset_chunks();
  layout_work(p);
  if (o.hbm_budget) {
    // shrink the chunked intermediates until the workspace fits; failing
    // that, keep the slab planes g, then also the spectra D, in host memory
    bool fits = shrink_to_budget(p, o.hbm_budget);
    for (int mode = 1; mode <= 2 && !fits; ++mode) {
      p->spill_g = true;
      p->spill_D = mode == 2;
      reset_chunks();
      fits = shrink_to_budget(p, o.hbm_budget);
    }
    if (!fits) {
      const size_t need = p->work_bytes;
      delete p;
      return fail(LAMINO_E_BUDGET,
                  "lamino_plan: workspace %zu bytes exceeds budget %zu even with the spectra and "
                  "slab planes in host memory",
                  need, o.hbm_budget);
    }
  }
  build_tables(p);
  p->d_tables = nullptr;
  p->d_work = nullptr;
  p->bound = false;
  p->profiling = false;
  for (int i = 0; i < LAMINO_NSTAGE; ++i) {
    p->stage_ms[i] = 0.0;
    p->stage_launches[i] = 0;
  }
  *out = p;
  return LAMINO_OK;
}

int lamino_plan_sizes(const lamino_plan_t* p, size_t* table_bytes, size_t* work_bytes) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_sizes: NULL plan");
  if (table_bytes) *table_bytes = p->table_bytes;
  if (work_bytes) *work_bytes = p->work_bytes;
  return LAMINO_OK;
}

int lamino_plan_info(const lamino_plan_t* p, lamino_info* info) {
  if (!p || !info) return fail(LAMINO_E_INVALID, "lamino_plan_info: NULL argument");
  info->h_p = p->h_p;
  info->w_p = p->w_p;
  info->n_slab = p->n_slab;
  info->grid = p->grid;
  info->kernel_m = p->M;
  info->beta = p->beta;
  info->z_chunk = p->z_chunk;
  info->slab_chunk = p->slab_chunk;
  info->theta_chunk = p->theta_chunk;
  info->table_bytes = p->table_bytes;
  info->work_bytes = p->work_bytes;
  info->off_spectra = p->off_D;
  info->bytes_spectra = p->bytes_D;
  info->off_slabs = p->off_g;
  info->spectra_scale = p->spectra_scale;
  info->bytes_slabs = p->bytes_g;
  info->spill_spectra = p->spill_D;
  info->spill_slabs = p->spill_g;
  info->col_chunk = p->col_chunk;
  info->io_z = p->io_z;
  info->host_bytes = p->host_bytes;
  info->io_bytes = p->io_bytes;
  return LAMINO_OK;
}

int lamino_plan_host_sizes(const lamino_plan_t* p, size_t* host_bytes, size_t* io_bytes) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_host_sizes: NULL plan");
  if (host_bytes) *host_bytes = p->host_bytes;
  if (io_bytes) *io_bytes = p->io_bytes;
  return LAMINO_OK;
}

int lamino_plan_bind_host(lamino_plan_t* p, void* h_spill) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_bind_host: NULL plan");
  if (p->host_bytes && !h_spill)
    return fail(LAMINO_E_INVALID, "lamino_plan_bind_host: the plan needs %zu bytes of host memory",
                p->host_bytes);
  if ((uintptr_t)h_spill & 255)
    return fail(LAMINO_E_INVALID, "lamino_plan_bind_host: buffer must be 256-byte aligned");
  p->h_spill = h_spill;
  return LAMINO_OK;
}

int lamino_plan_bind(lamino_plan_t* p, void* d_tables, void* d_work, void* stream) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_bind: NULL plan");
  if (!d_tables || !d_work) return fail(LAMINO_E_INVALID, "lamino_plan_bind: NULL buffer");
  if (((uintptr_t)d_tables & 255) || ((uintptr_t)d_work & 255))
    return fail(LAMINO_E_INVALID, "lamino_plan_bind: buffers must be 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(d_tables, p->host_tables.data(), p->table_bytes,
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "lamino_plan_bind: table upload");
  // the host staging copy must stay valid until the copy has run
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "lamino_plan_bind: synchronise");
  p->d_tables = d_tables;
  p->d_work = d_work;
  p->bound = true;
  return LAMINO_OK;
}

int lamino_plan_table_image(const lamino_plan_t* p, void* host_dst, size_t bytes) {
  if (!p || !host_dst) return fail(LAMINO_E_INVALID, "lamino_plan_table_image: NULL argument");
  if (bytes < p->table_bytes)
    return fail(LAMINO_E_INVALID, "lamino_plan_table_image: %zu bytes given, %zu needed", bytes,
                p->table_bytes);
  std::memcpy(host_dst, p->host_tables.data(), p->table_bytes);
  return LAMINO_OK;
}

int lamino_plan_attach(lamino_plan_t* p, void* d_tables, void* d_work) {
  if (!p) return fail(LAMINO_E_INVALID, "lamino_plan_attach: NULL plan");
  if (!d_tables || !d_work) return fail(LAMINO_E_INVALID, "lamino_plan_attach: NULL buffer");
  if (((uintptr_t)d_tables & 255) || ((uintptr_t)d_work & 255))
    return fail(LAMINO_E_INVALID, "lamino_plan_attach: buffers must be 256-byte aligned");
  p->d_tables = d_tables;
  p->d_work = d_work;
  p->bound = true;
  return LAMINO_OK;
}

static int check_call(const lamino_plan_t* p, const void* a, const void* b, const char* who) {
  if (!p) return fail(LAMINO_E_INVALID, "%s: NULL plan", who);
  if (!p->bound) return fail(LAMINO_E_UNBOUND, "%s: plan is not bound", who);
  if (!a || !b) return fail(LAMINO_E_INVALID, "%s: NULL data or volume pointer", who);
  if (p->host_bytes && !p->h_spill)
    return fail(LAMINO_E_UNBOUND, "%s: the plan keeps intermediates in host memory and no host "
                "buffer is bound (lamino_plan_bind_host)", who);
  return LAMINO_OK;
}

// Operations that need the spectra and slab planes on the device.
static int check_resident(const lamino_plan_t* p, const char* who) {
  if (p->spill_D || p->spill_g)
    return fail(LAMINO_E_UNSUPPORTED, "%s: not available for a plan whose intermediates live in "
                "host memory (raise opts.hbm_budget)", who);
  return LAMINO_OK;
}

int lamino_fbp_host(const lamino_plan_t* p, const void* h_data, float* h_vol, void* d_io,
                    void* stream) {
  const int c = check_call(p, h_data, h_vol, "lamino_fbp_host");
  if (c) return c;
  if (!d_io) return fail(LAMINO_E_INVALID, "lamino_fbp_host: NULL staging buffer");
  if ((uintptr_t)d_io & 255)
    return fail(LAMINO_E_INVALID, "lamino_fbp_host: staging buffer must be 256-byte aligned");
  lam::BackprojOpts o;
  o.h_data = h_data;
  o.h_vol = h_vol;
  o.io = d_io;
  hipError_t e = lam::run_backprojection(p, nullptr, nullptr, true, static_cast<hipStream_t>(stream), o);
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_fbp_host");
}

int lamino_fbp(const lamino_plan_t* p, const void* d_data, float* d_vol, void* stream) {
  const int c = check_call(p, d_data, d_vol, "lamino_fbp");
  if (c) return c;
  hipError_t e = lam::run_backprojection(p, d_data, d_vol, true, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_fbp");
}

int lamino_fbp_raw(const lamino_plan_t* p, const void* d_raw, const float* d_dark,
                   const float* d_flat, double min_ratio, float* d_vol, void* stream) {
  const int c = check_call(p, d_raw, d_vol, "lamino_fbp_raw");
  if (c) return c;
  if (!d_dark || !d_flat) return fail(LAMINO_E_INVALID, "lamino_fbp_raw: NULL dark or flat field");
  if (!std::isfinite(min_ratio) || !(min_ratio > 0.0) || (float)min_ratio <= 0.f)
    return fail(LAMINO_E_INVALID, "lamino_fbp_raw: min_ratio must be a positive float");
  lam::BackprojOpts o;
  o.dark = d_dark;
  o.flat = d_flat;
  o.min_ratio = (float)min_ratio;
  hipError_t e = lam::run_backprojection(p, d_raw, d_vol, true, static_cast<hipStream_t>(stream), o);
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_fbp_raw");
}

int lamino_fbp_slices(const lamino_plan_t* p, const void* d_data, double center_shift, int z_first,
                      int z_count, float* d_out, void* stream) {
  const int c = check_call(p, d_data, d_out, "lamino_fbp_slices");
  if (c) return c;
  if (z_first < 0 || z_count < 1 || z_first > p->nz - z_count)
    return fail(LAMINO_E_INVALID, "lamino_fbp_slices: slices [%d, %d + %d) outside [0, %d)", z_first,
                z_first, z_count, p->nz);
  const double room = 0.5 * (p->w_p - p->w);
  if (!std::isfinite(center_shift) || std::fabs(center_shift) > room)
    return fail(LAMINO_E_INVALID, "lamino_fbp_slices: |center_shift| must be <= (w_p - w) / 2 = %g",
                room);
  lam::BackprojOpts o;
  o.center_shift = center_shift;
  o.z_first = z_first;
  o.z_count = z_count;
  hipError_t e = lam::run_backprojection(p, d_data, d_out, true, static_cast<hipStream_t>(stream), o);
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_fbp_slices");
}

int lamino_adj(const lamino_plan_t* p, const void* d_data, float* d_vol, void* stream) {
  const int c = check_call(p, d_data, d_vol, "lamino_adj");
  if (c) return c;
  hipError_t e = lam::run_backprojection(p, d_data, d_vol, false, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_adj");
}

int lamino_fwd(const lamino_plan_t* p, const float* d_vol, void* d_data, void* stream) {
  int c = check_call(p, d_vol, d_data, "lamino_fwd");
  if (c) return c;
  c = check_resident(p, "lamino_fwd");
  if (c) return c;
  if (lam::integer_dtype(p->opts.data_dtype))
    return fail(LAMINO_E_INVALID, "lamino_fwd: integer data is accepted as input only");
  hipError_t e = lam::run_forward(p, d_vol, d_data, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_fwd");
}

int lamino_direct_work_bytes(const lamino_plan_t* p, size_t* bytes) {
  if (!p || !bytes) return fail(LAMINO_E_INVALID, "lamino_direct_work_bytes: NULL argument");
  *bytes = lam::direct_work_bytes(p);
  return LAMINO_OK;
}

int lamino_direct_fbp(const lamino_plan_t* p, const void* d_data, float* d_vol, void* d_work,
                      void* stream) {
  const int c = check_call(p, d_data, d_vol, "lamino_direct_fbp");
  if (c) return c;
  if (!d_work) return fail(LAMINO_E_INVALID, "lamino_direct_fbp: NULL workspace");
  if ((uintptr_t)d_work & 255)
    return fail(LAMINO_E_INVALID, "lamino_direct_fbp: workspace must be 256-byte aligned");
  hipError_t e = lam::run_direct(p, d_data, d_vol, d_work, true, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_direct_fbp");
}

int lamino_direct_adj(const lamino_plan_t* p, const void* d_data, float* d_vol, void* stream) {
  const int c = check_call(p, d_data, d_vol, "lamino_direct_adj");
  if (c) return c;
  hipError_t e = lam::run_direct(p, d_data, d_vol, nullptr, false, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_direct_adj");
}

static int check_tv(const void* a, const void* b, int nz, int ny, int nx, const char* who) {
  if (!a || !b) return fail(LAMINO_E_INVALID, "%s: NULL pointer", who);
  if (nz <= 0 || ny <= 0 || nx <= 0)
    return fail(LAMINO_E_INVALID, "%s: sizes must be positive (%d, %d, %d)", who, nz, ny, nx);
  if (!lam::tv_dims_ok(nz, ny, nx))
    return fail(LAMINO_E_UNSUPPORTED, "%s: volume %d x %d x %d too large", who, nz, ny, nx);
  return LAMINO_OK;
}

static bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int lamino_tv_grad(const float* d_vol, float* d_grad, int nz, int ny, int nx, void* stream) {
  const int c = check_tv(d_vol, d_grad, nz, ny, nx, "lamino_tv_grad");
  if (c) return c;
  hipError_t e = lam::tv_grad(d_vol, d_grad, nz, ny, nx, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_tv_grad");
}

int lamino_tv_div(const float* d_p, float* d_out, int nz, int ny, int nx, void* stream) {
  const int c = check_tv(d_p, d_out, nz, ny, nx, "lamino_tv_div");
  if (c) return c;
  hipError_t e = lam::tv_div(d_p, d_out, nz, ny, nx, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_tv_div");
}

int lamino_tv_term(const float* d_vol, const float* d_shift, const float* d_base, double rho,
                   float* d_out, int nz, int ny, int nx, void* stream) {
  const int c = check_tv(d_vol, d_out, nz, ny, nx, "lamino_tv_term");
  if (c) return c;
  if (!std::isfinite(rho)) return fail(LAMINO_E_INVALID, "lamino_tv_term: rho must be finite");
  hipError_t e = lam::tv_term(d_vol, d_shift, d_base, (float)rho, d_out, nz, ny, nx,
                              static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_tv_term");
}

int lamino_tv_shrink(const float* d_vol, float* d_lambda, float* d_shift, float* d_psi,
                     double alpha, double rho, int nz, int ny, int nx, void* stream) {
  int c = check_tv(d_vol, d_lambda, nz, ny, nx, "lamino_tv_shrink");
  if (c) return c;
  if (!d_shift) return fail(LAMINO_E_INVALID, "lamino_tv_shrink: NULL shift");
  if (!finite_pos(rho) || !std::isfinite(alpha) || alpha < 0.0)
    return fail(LAMINO_E_INVALID, "lamino_tv_shrink: need rho > 0 and alpha >= 0 (finite)");
  hipError_t e = lam::tv_shrink(d_vol, d_lambda, d_shift, d_psi, (float)alpha, (float)rho, nz, ny,
                                nx, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_tv_shrink");
}

int lamino_admm_tv_state_bytes(const lamino_plan_t* p, size_t* bytes) {
  if (!p || !bytes) return fail(LAMINO_E_INVALID, "lamino_admm_tv_state_bytes: NULL argument");
  if (!lam::tv_dims_ok(p->nz, p->n, p->n))
    return fail(LAMINO_E_UNSUPPORTED, "lamino_admm_tv_state_bytes: volume too large");
  *bytes = lam::admm_state_bytes(p);
  return LAMINO_OK;
}

int lamino_admm_tv(const lamino_plan_t* p, const float* d_data, float* d_vol, double alpha,
                   double rho, int outer, int inner, int resume, void* d_state, void* stream) {
  int c = check_call(p, d_data, d_vol, "lamino_admm_tv");
  if (c) return c;
  c = check_resident(p, "lamino_admm_tv");
  if (c) return c;
  if (!d_state) return fail(LAMINO_E_INVALID, "lamino_admm_tv: NULL state");
  if ((uintptr_t)d_state & 255)
    return fail(LAMINO_E_INVALID, "lamino_admm_tv: state must be 256-byte aligned");
  if (p->opts.data_dtype != LAMINO_F32)
    return fail(LAMINO_E_INVALID, "lamino_admm_tv: the plan's data dtype must be float32");
  if (!finite_pos(rho) || !std::isfinite(alpha) || alpha < 0.0)
    return fail(LAMINO_E_INVALID, "lamino_admm_tv: need rho > 0 and alpha >= 0 (finite)");
  if (outer < 0 || inner < 0)
    return fail(LAMINO_E_INVALID, "lamino_admm_tv: negative iteration count");
  if (!lam::tv_dims_ok(p->nz, p->n, p->n))
    return fail(LAMINO_E_UNSUPPORTED, "lamino_admm_tv: volume too large");
  hipError_t e = lam::run_admm_tv(p, d_data, d_vol, (float)alpha, (float)rho, outer, inner,
                                  resume, d_state, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? LAMINO_OK : hip_fail(e, "lamino_admm_tv");
}

int lamino_plan_destroy(lamino_plan_t* p) {
  if (!p) return LAMINO_OK;
  for (hipEvent_t e : p->ev)
    if (e) (void)hipEventDestroy(e);
  if (p->s_in) (void)hipStreamDestroy(p->s_in);
  if (p->s_out) (void)hipStreamDestroy(p->s_out);
  for (auto& m : p->marks) {
    (void)hipEventSynchronize(m.stop);
    (void)hipEventDestroy(m.start);
    (void)hipEventDestroy(m.stop);
  }
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  delete p;
  return LAMINO_OK;
}

const char* lamino_strerror(int status) {
  switch (status) {
    case LAMINO_OK: return "success";
    case LAMINO_E_INVALID: return "invalid argument";
    case LAMINO_E_UNSUPPORTED: return "unsupported size";
    case LAMINO_E_BUDGET: return "workspace exceeds the memory budget";
    case LAMINO_E_HIP: return "HIP runtime error";
    case LAMINO_E_UNBOUND: return "plan not bound to device buffers";
    default: return "unknown status";
  }
}

const char* lamino_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
