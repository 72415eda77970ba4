"""ctypes binding of include/lamino.h (argument marshalling only).

Every function here has the name of the C entry point it calls.  The
library is loaded from the package's `lib/liblamino.so`; a missing
library is an error (there is no fallback implementation).
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "liblamino.so")

LAMINO_F32, LAMINO_F16, LAMINO_BF16, LAMINO_U8, LAMINO_U16 = 0, 1, 2, 3, 4
LAMINO_RAMP, LAMINO_SHEPP_LOGAN, LAMINO_PARZEN = 0, 1, 2
LAMINO_OK = 0
LAMINO_E_INVALID = -1
LAMINO_E_UNSUPPORTED = -2
LAMINO_E_BUDGET = -3
LAMINO_E_HIP = -4
LAMINO_E_UNBOUND = -5

EXPORTED = (
    "lamino_opts_default",
    "lamino_plan",
    "lamino_plan_sizes",
    "lamino_plan_info",
    "lamino_plan_bind",
    "lamino_plan_host_sizes",
    "lamino_plan_bind_host",
    "lamino_fbp_host",
    "lamino_plan_table_image",
    "lamino_plan_attach",
    "lamino_fbp",
    "lamino_fbp_raw",
    "lamino_fbp_slices",
    "lamino_fwd",
    "lamino_adj",
    "lamino_plan_profile",
    "lamino_plan_stage_times",
    "lamino_plan_destroy",
    "lamino_strerror",
    "lamino_last_error",
    "lamino_direct_work_bytes",
    "lamino_direct_fbp",
    "lamino_direct_adj",
    "lamino_tv_grad",
    "lamino_tv_div",
    "lamino_tv_term",
    "lamino_tv_shrink",
    "lamino_admm_tv_state_bytes",
    "lamino_admm_tv",
    "lamino_fbp_noalloc",
)


class lamino_geom(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int),
        ("n", ctypes.c_int),
        ("n_theta", ctypes.c_int),
        ("h", ctypes.c_int),
        ("w", ctypes.c_int),
        ("tilt", ctypes.c_double),
        ("theta", ctypes.POINTER(ctypes.c_double)),
    ]


class lamino_opts(ctypes.Structure):
    _fields_ = [
        ("data_dtype", ctypes.c_int),
        ("storage_dtype", ctypes.c_int),
        ("filter", ctypes.c_int),
        ("pad_u", ctypes.c_double),
        ("pad_v", ctypes.c_double),
        ("kernel_m", ctypes.c_int),
        ("z_chunk", ctypes.c_int),
        ("slab_chunk", ctypes.c_int),
        ("theta_chunk", ctypes.c_int),
        ("hbm_budget", ctypes.c_size_t),
    ]


class lamino_info(ctypes.Structure):
    _fields_ = [
        ("h_p", ctypes.c_int),
        ("w_p", ctypes.c_int),
        ("n_slab", ctypes.c_int),
        ("grid", ctypes.c_int),
        ("kernel_m", ctypes.c_int),
        ("beta", ctypes.c_double),
        ("z_chunk", ctypes.c_int),
        ("slab_chunk", ctypes.c_int),
        ("theta_chunk", ctypes.c_int),
        ("table_bytes", ctypes.c_size_t),
        ("work_bytes", ctypes.c_size_t),
        ("off_spectra", ctypes.c_size_t),
        ("bytes_spectra", ctypes.c_size_t),
        ("off_slabs", ctypes.c_size_t),
        ("bytes_slabs", ctypes.c_size_t),
        ("spectra_scale", ctypes.c_double),
        ("spill_spectra", ctypes.c_int),
        ("spill_slabs", ctypes.c_int),
        ("col_chunk", ctypes.c_int),
        ("io_z", ctypes.c_int),
        ("host_bytes", ctypes.c_size_t),
        ("io_bytes", ctypes.c_size_t),
    ]


class LaminoError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lamino_last_error() or lamino_strerror(code)
        super().__init__(f"{where} failed ({code}: {lamino_strerror(code)}): {msg}")


_lib = None


def load_library(path=LIB_PATH):
    """Load liblamino.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} not found: build it with `python -m paper_2401_11101_amd.build` "
            "(the HIP library is required; there is no fallback)"
        )
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.lamino_opts_default.argtypes = [ctypes.POINTER(lamino_opts)]
    lib.lamino_opts_default.restype = None
    lib.lamino_plan.argtypes = [ctypes.POINTER(lamino_geom), ctypes.POINTER(lamino_opts), ctypes.POINTER(P)]
    lib.lamino_plan_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.lamino_plan_info.argtypes = [P, ctypes.POINTER(lamino_info)]
    lib.lamino_plan_bind.argtypes = [P, P, P, P]
    lib.lamino_plan_table_image.argtypes = [P, P, ctypes.c_size_t]
    lib.lamino_plan_host_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.lamino_plan_bind_host.argtypes = [P, P]
    lib.lamino_fbp_host.argtypes = [P, P, P, P, P]
    lib.lamino_plan_attach.argtypes = [P, P, P]
    lib.lamino_fbp.argtypes = [P, P, P, P]
    lib.lamino_fwd.argtypes = [P, P, P, P]
    lib.lamino_adj.argtypes = [P, P, P, P]
    lib.lamino_plan_profile.argtypes = [P, ctypes.c_int]
    lib.lamino_plan_stage_times.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    lib.lamino_plan_destroy.argtypes = [P]
    lib.lamino_strerror.argtypes = [ctypes.c_int]
    lib.lamino_strerror.restype = ctypes.c_char_p
    lib.lamino_last_error.argtypes = []
    lib.lamino_last_error.restype = ctypes.c_char_p
    I, D = ctypes.c_int, ctypes.c_double
    lib.lamino_fbp_raw.argtypes = [P, P, P, P, D, P, P]
    lib.lamino_fbp_slices.argtypes = [P, P, D, I, I, P, P]
    lib.lamino_direct_work_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.lamino_direct_fbp.argtypes = [P, P, P, P, P]
    lib.lamino_direct_adj.argtypes = [P, P, P, P]
    lib.lamino_tv_grad.argtypes = [P, P, I, I, I, P]
    lib.lamino_tv_div.argtypes = [P, P, I, I, I, P]
    lib.lamino_tv_term.argtypes = [P, P, P, D, P, I, I, I, P]
    lib.lamino_tv_shrink.argtypes = [P, P, P, P, D, D, I, I, I, P]
    lib.lamino_admm_tv_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    lib.lamino_admm_tv.argtypes = [P, P, P, D, D, I, I, I, P, P]
    lib.lamino_fbp_noalloc.argtypes = [P, P, P, P]
    for name in ("lamino_plan", "lamino_plan_sizes", "lamino_plan_info", "lamino_plan_bind",
                 "lamino_plan_table_image", "lamino_plan_attach", "lamino_plan_host_sizes",
                 "lamino_plan_bind_host", "lamino_fbp_host",
                 "lamino_fbp", "lamino_fwd", "lamino_adj", "lamino_plan_destroy",
                 "lamino_plan_profile", "lamino_plan_stage_times", "lamino_tv_grad",
                 "lamino_tv_div", "lamino_tv_term", "lamino_tv_shrink", "lamino_direct_work_bytes",
                 "lamino_direct_fbp", "lamino_direct_adj", "lamino_fbp_raw", "lamino_fbp_slices",
                 "lamino_admm_tv_state_bytes", "lamino_admm_tv", "lamino_fbp_noalloc"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(code, where):
    if code != LAMINO_OK:
        raise LaminoError(code, where)


def lamino_opts_default():
    o = lamino_opts()
    load_library().lamino_opts_default(ctypes.byref(o))
    return o


def lamino_plan(geom, opts):
    """Returns an opaque plan handle (c_void_p)."""
    h = ctypes.c_void_p()
    _check(load_library().lamino_plan(ctypes.byref(geom), ctypes.byref(opts), ctypes.byref(h)), "lamino_plan")
    return h


def lamino_plan_sizes(plan):
    t, w = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().lamino_plan_sizes(plan, ctypes.byref(t), ctypes.byref(w)), "lamino_plan_sizes")
    return t.value, w.value


def lamino_plan_info(plan):
    info = lamino_info()
    _check(load_library().lamino_plan_info(plan, ctypes.byref(info)), "lamino_plan_info")
    return info


def lamino_plan_bind(plan, d_tables, d_work, stream):
    _check(load_library().lamino_plan_bind(plan, d_tables, d_work, stream), "lamino_plan_bind")


def lamino_plan_host_sizes(plan):
    """(host_bytes, io_bytes) of an out-of-core plan."""
    hb, io = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load_library().lamino_plan_host_sizes(plan, ctypes.byref(hb), ctypes.byref(io)),
           "lamino_plan_host_sizes")
    return hb.value, io.value


def lamino_plan_bind_host(plan, h_spill):
    _check(load_library().lamino_plan_bind_host(plan, h_spill), "lamino_plan_bind_host")


def lamino_fbp_host(plan, h_data, h_vol, d_io, stream):
    _check(load_library().lamino_fbp_host(plan, h_data, h_vol, d_io, stream), "lamino_fbp_host")


def lamino_plan_table_image(plan, host_dst, nbytes):
    _check(load_library().lamino_plan_table_image(plan, host_dst, nbytes), "lamino_plan_table_image")


def lamino_plan_attach(plan, d_tables, d_work):
    _check(load_library().lamino_plan_attach(plan, d_tables, d_work), "lamino_plan_attach")


def lamino_fbp(plan, d_data, d_vol, stream):
    _check(load_library().lamino_fbp(plan, d_data, d_vol, stream), "lamino_fbp")


def lamino_fbp_raw(plan, d_raw, d_dark, d_flat, min_ratio, d_vol, stream):
    _check(load_library().lamino_fbp_raw(plan, d_raw, d_dark, d_flat, float(min_ratio), d_vol, stream),
           "lamino_fbp_raw")


def lamino_fbp_slices(plan, d_data, center_shift, z_first, z_count, d_out, stream):
    _check(load_library().lamino_fbp_slices(plan, d_data, float(center_shift), int(z_first),
                                            int(z_count), d_out, stream), "lamino_fbp_slices")


def lamino_fwd(plan, d_vol, d_data, stream):
    _check(load_library().lamino_fwd(plan, d_vol, d_data, stream), "lamino_fwd")


def lamino_adj(plan, d_data, d_vol, stream):
    _check(load_library().lamino_adj(plan, d_data, d_vol, stream), "lamino_adj")


def lamino_direct_work_bytes(plan):
    b = ctypes.c_size_t()
    _check(load_library().lamino_direct_work_bytes(plan, ctypes.byref(b)), "lamino_direct_work_bytes")
    return b.value


def lamino_direct_fbp(plan, d_data, d_vol, d_work, stream):
    _check(load_library().lamino_direct_fbp(plan, d_data, d_vol, d_work, stream), "lamino_direct_fbp")


def lamino_direct_adj(plan, d_data, d_vol, stream):
    _check(load_library().lamino_direct_adj(plan, d_data, d_vol, stream), "lamino_direct_adj")


def lamino_tv_grad(d_vol, d_grad, nz, ny, nx, stream):
    _check(load_library().lamino_tv_grad(d_vol, d_grad, nz, ny, nx, stream), "lamino_tv_grad")


def lamino_tv_div(d_p, d_out, nz, ny, nx, stream):
    _check(load_library().lamino_tv_div(d_p, d_out, nz, ny, nx, stream), "lamino_tv_div")


def lamino_tv_term(d_vol, d_shift, d_base, rho, d_out, nz, ny, nx, stream):
    _check(load_library().lamino_tv_term(d_vol, d_shift, d_base, float(rho), d_out, nz, ny, nx,
                                         stream), "lamino_tv_term")


def lamino_tv_shrink(d_vol, d_lambda, d_shift, d_psi, alpha, rho, nz, ny, nx, stream):
    _check(load_library().lamino_tv_shrink(d_vol, d_lambda, d_shift, d_psi, float(alpha),
                                           float(rho), nz, ny, nx, stream), "lamino_tv_shrink")


def lamino_admm_tv_state_bytes(plan):
    b = ctypes.c_size_t()
    _check(load_library().lamino_admm_tv_state_bytes(plan, ctypes.byref(b)),
           "lamino_admm_tv_state_bytes")
    return b.value


def lamino_admm_tv(plan, d_data, d_vol, alpha, rho, outer, inner, resume, d_state, stream):
    _check(load_library().lamino_admm_tv(plan, d_data, d_vol, float(alpha), float(rho), int(outer),
                                         int(inner), int(bool(resume)), d_state, stream),
           "lamino_admm_tv")


NSTAGE = 4
STAGE_NAMES = ("detector", "gridding", "slab", "x3")


def lamino_plan_profile(plan, enable):
    _check(load_library().lamino_plan_profile(plan, int(bool(enable))), "lamino_plan_profile")


def lamino_plan_stage_times(plan, reset=False):
    """{stage: (milliseconds, launches)} accumulated while profiling was on."""
    ms = (ctypes.c_double * NSTAGE)()
    n = (ctypes.c_int * NSTAGE)()
    _check(load_library().lamino_plan_stage_times(plan, ms, n, int(bool(reset))), "lamino_plan_stage_times")
    return {STAGE_NAMES[i]: (ms[i], n[i]) for i in range(NSTAGE)}


def lamino_plan_destroy(plan):
    if plan:
        load_library().lamino_plan_destroy(plan)


def lamino_strerror(code):
    return load_library().lamino_strerror(code).decode()


def lamino_last_error():
    return load_library().lamino_last_error().decode()


# device scratch of lamino_fbp_noalloc (LAMINO_SCRATCH_BYTES in lamino.h)
LAMINO_SCRATCH_BYTES = 64 << 20


def lamino_fbp_noalloc(plan, d_data, d_vol, stream):
    _check(load_library().lamino_fbp_noalloc(plan, d_data, d_vol, stream), "lamino_fbp_noalloc")
