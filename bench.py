"""Benchmark: GVoxel/s of the Fourier-route FBP on one MI355X.

Workload: volume 256 x 256 x 256, 400 projections over [0, 2 pi), tilt
25 deg, detector 256 x 256, 50 seeded ellipsoids, float32 data with 0.5%
Gaussian noise (exact projections computed on the GPU from the closed
form; the paper's datasets are not available).  A step is one FBP of the
whole batch with inputs resident in HBM.  The float32 path (storage f32,
Gaussian half-width 5) gives `value`; the fp16-storage path (half-width
3) is reported beside it, with the forward and adjoint operators.

Per-stage device times come from HIP events that the library records on
the call stream during the timed steps; `roofline` reports the dominant
kernel against MI355X peaks.  `cpu_baseline` times the CPU FP64 oracle's
Gaussian-USFFT FBP on a bounded sample of frequency slabs (rank 0, N=1).

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import synth  # noqa: E402

NZ = N = H = W = 256
NT = 400
TILT = np.deg2rad(25.0)
HBM_PEAK_GBS = 8000.0
MFMA_BF16_PEAK_TFLOPS = 2500.0
FP32_VECTOR_PEAK_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_data(device):
    ells = synth.random_ellipsoids(50, NZ, N, seed=0)
    d = synth.project_ellipsoids(ells, NT, H, W, TILT, device=device, dtype=torch.float64)
    d = synth.add_noise(d, 0.005, seed=1)
    return d.float().contiguous()


def time_op(fn, steps, warmup, stream, plan=None):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    if plan is not None:
        plan.stage_times(reset=True)
        plan.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    stages = None
    if plan is not None:
        plan.profile(False)
        stages = plan.stage_times(reset=True)
    return ev0.elapsed_time(ev1) / steps, wall, stages


def algorithmic_work(info, storage_bytes, data_bytes):
    """Algorithmic bytes / flops per FBP of each stage: reads and writes that
    the stage must make once (input, output and the chunked intermediates it
    owns), and 5 flops per Gaussian tap / 4 per x3 multiply-add."""
    n_slab, w_p, grid, M = info.n_slab, info.w_p, info.grid, info.kernel_m
    samples = n_slab * NT * (w_p - 1)
    return {
        # read d, write D
        "detector": {"bytes": NT * H * W * data_bytes + n_slab * NT * w_p * storage_bytes},
        # read D, write the slab grids; 5 flops per tap
        "gridding": {"bytes": n_slab * NT * w_p * storage_bytes + n_slab * grid * grid * 8,
                     "flops": 5.0 * (2 * M) ** 2 * samples},
        # read the slab grids, write g
        "slab": {"bytes": n_slab * grid * grid * 8 + n_slab * N * N * storage_bytes},
        # read g, write vol; 4 flops per (z, l, column)
        "x3": {"bytes": n_slab * N * N * storage_bytes + NZ * N * N * 4,
               "flops": 4.0 * NZ * n_slab * N * N},
    }


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fbp_256cube_400proj_hbm_traffic.md")
STATS_FILE = os.path.join(ROOT, "profiles", "fbp_256cube_400proj_kernel_stats.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2401_11101_amd", "csrc", f)
                  for f in ("lamino_kernels.hip", "lamino_common.h", "lamino_device.h")]


def _sources_hash():
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_figure(path, tag, kernel):
    """A figure recorded in a committed profile summary as
    <!-- tag kernel=K value=V source=S -->, or None when the kernel sources
    changed after it was taken."""
    import re

    try:
        text = open(path).read()
    except OSError:
        return None
    for m in re.finditer(rf"<!-- {tag} kernel=(.+?) value=([0-9.eE+-]+) source=([0-9a-f]+) -->", text):
        if m.group(1) == kernel and m.group(3) == _sources_hash():
            return float(m.group(2))
    return None


def roofline(stages, work, steps, info):
    """Dominant stage against its peak: algorithmic work per launch (work per
    FBP / launches per FBP) over the mean launch duration from the events."""
    name = max(stages, key=lambda k: stages[k][0])
    ms, launches = stages[name]
    per_launch_ms = ms / max(launches, 1)
    per_fbp = max(launches, 1) / steps
    w = work[name]
    if name == "gridding":
        kernel = f"k_spread<{info.kernel_m}, 0>"
        # matrix-core gridding: algorithmic taps as float32 vector work
        achieved = w["flops"] / per_fbp / (per_launch_ms * 1e-3) / 1e12
        # the same taps as bf16 matrix-core products: a complex value times a
        # real weight is 2 real products, each formed from 3 bf16 products
        # (hi hi, hi lo, lo hi), 2 flops each
        mfma = 12.0 / 5.0 * achieved
        rp = _profile_figure(STATS_FILE, "stats", kernel)
        traffic = _profile_figure(TRAFFIC_FILE, "traffic", kernel)
        return {"kernel": f"{kernel} (gridding)", "bound": "alu", "achieved": round(achieved, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": int(traffic) if traffic is not None else None,
                "algorithmic_bytes": w["bytes"],
                "launch_ms_events": round(per_launch_ms, 4),
                "launch_ms_rocprof": round(rp / 1e3, 4) if rp is not None else None,
                "mfma_view": {"achieved": round(mfma, 2), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": round(mfma / MFMA_BF16_PEAK_TFLOPS, 5),
                              "note": "useful bf16 products of the taps (12 flops per tap)"}}
    achieved = w["bytes"] / per_fbp / (per_launch_ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
            "launch_ms_events": round(per_launch_ms, 4)}


def _pool_workers():
    """Host processes for the CPU legs: the host's CPU share (at most 16)."""
    return max(1, min(16, os.cpu_count() or 1))


def _o3_slab(args):
    """One frequency slab of oracle O3 (Gaussian USFFT, M = 12): gridding,
    inverse FFT and psi correction, then its x3 contribution to the whole
    volume; returns a checksum so that nothing is skipped."""
    from threadpoolctl import threadpool_limits

    from oracle import nudft, usfft
    from oracle.geometry import Geometry, freqs

    l, Gl, geo = args
    with threadpool_limits(1):
        g = Geometry(**geo)
        N_g = usfft.default_grid(g.n)
        X, Y = usfft.slab_positions(g, l, N_g)
        gl = usfft.type1(Gl, X, Y, g.n, N_g, 12)
        E = nudft.x3_phases(g, +1.0)[:, int(np.where(freqs(g.h_p) == l)[0][0])]
        acc = np.real(E[:, None, None] * gl[None])
        return float(acc.sum())


def _exact_columns(args):
    """Exact Fourier FBP sums (oracle O2) of the columns (ys, xs) over the
    frequency slabs ls: sum_l E(x3, l) g_l(column), complex.  The data come
    from a .npy file; their spectra are formed 16 projections at a time."""
    from threadpoolctl import threadpool_limits

    from oracle import filters, nudft
    from oracle.geometry import Geometry, freqs

    path, ls, geo, ys, xs = args
    with threadpool_limits(1):
        g = Geometry(**geo)
        d = np.load(path, mmap_mode="r")
        all_ls = freqs(g.h_p)
        li = np.array([int(np.where(all_ls == l)[0][0]) for l in ls])
        ms = freqs(g.w_p)
        x1 = np.asarray(xs) - g.n // 2
        x2 = np.asarray(ys) - g.n // 2
        ku = (ms / g.w_p)[None, :]
        E = nudft.x3_phases(g, +1.0)
        gl = np.zeros((len(ls), len(xs)), dtype=np.complex128)
        for t0 in range(0, g.n_theta, 16):
            th = g.theta[t0:t0 + 16]
            gs = Geometry(nz=g.nz, n=g.n, n_theta=len(th), h=g.h, w=g.w, phi=g.phi, theta=th)
            G = nudft.filter_spectra(nudft.data_spectra_fft(np.asarray(d[t0:t0 + 16]), gs), g,
                                     filters.SHEPP_LOGAN)[:, li, :]
            ct, st = np.cos(th)[:, None], np.sin(th)[:, None]
            for k, l in enumerate(ls):
                kv = l / g.h_p
                xi1 = (ku * ct + kv * st * np.sin(g.phi)).reshape(-1)
                xi2 = (ku * st - kv * ct * np.sin(g.phi)).reshape(-1)
                ph = np.exp(2j * np.pi * (np.outer(xi1, x1) + np.outer(xi2, x2)))
                gl[k] += G[:, k, :].reshape(-1) @ ph
        return E[:, li] @ gl


def cpu_baseline(data_np, vols, slabs_per_run=None, runs=3):
    """The CPU oracle on the GPU host, on a bounded sample of the workload.

    Timing: oracle O3 (FP64 Gaussian-USFFT FBP, numpy) with the host's cores
    in a process pool: the detector transform and filter of all projections
    (numpy's FFT, one process), then a sample of frequency slabs spread over
    the spectrum, one slab per task, gridded and x3-accumulated in parallel;
    the whole FBP is extrapolated from the mean slab time.  Median of `runs`.

    Accuracy: the exact FP64 Fourier sums (oracle O2) on sampled volume
    columns against the GPU volumes `vols` ({name: volume}), relative L2."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    from oracle import filters, nudft
    from oracle.geometry import Geometry, freqs

    g = Geometry(nz=NZ, n=N, n_theta=NT, h=H, w=W, phi=TILT)
    geo = dict(nz=NZ, n=N, n_theta=NT, h=H, w=W, phi=TILT)
    workers = _pool_workers()
    slabs_per_run = slabs_per_run or 2 * workers
    half = g.h_p // 2
    ls_all = freqs(g.h_p)
    totals = []
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as pool:
        list(pool.map(_o3_slab, [(0, np.zeros(NT * (g.w_p - 1), complex), geo)] * workers))  # warm
        for r in range(runs):
            t0 = time.perf_counter()
            Gs = nudft.filter_spectra(nudft.data_spectra_fft(data_np, g, half=True), g,
                                      filters.SHEPP_LOGAN)
            t_det = time.perf_counter() - t0
            order = [((k + r * slabs_per_run) * 97) % half for k in range(slabs_per_run)]
            t1 = time.perf_counter()
            list(pool.map(_o3_slab, [(l, Gs[:, l, :].reshape(-1), geo) for l in order]))
            t_slabs = time.perf_counter() - t1
            totals.append(t_det + t_slabs / slabs_per_run * len(ls_all))
            del Gs
        t_total = float(np.median(totals))
        # exact sums on sampled columns against the GPU volumes
        ys = np.array([0, 77, 128, 201])
        xs = np.array([3, 128, 64, 250])
        import tempfile

        with tempfile.TemporaryDirectory() as tmp:
            path = os.path.join(tmp, "data.npy")
            np.save(path, data_np)
            parts = np.array_split(ls_all, workers)
            ref = sum(pool.map(_exact_columns, [(path, part, geo, ys, xs) for part in parts])).real
    rel = {name: float(np.linalg.norm(v[:, ys, xs].astype(np.float64) - ref) / np.linalg.norm(ref))
           for name, v in vols.items()}
    base = {"value": round(NZ * N * N / t_total / 1e9, 9), "unit": "GVoxel/s", "cores": workers,
            "kind": "oracle",
            "sample": f"O3 FP64 Gaussian-USFFT FBP (numpy, M=12): detector FFT + filter of all {NT} "
                      f"projections (one process) and {slabs_per_run} of the {len(ls_all)} frequency "
                      f"slabs it grids (all angles; one slab per task on {workers} processes), "
                      f"scaled linearly to the whole 256^3 FBP; median of {runs} runs "
                      f"({', '.join(f'{t:.0f}' for t in totals)} s extrapolated)"}
    return base, {"columns": [[int(y), int(x)] for y, x in zip(ys, xs)], "rel_l2": rel}


def cpu_direct_fbp(data_np, budget_s=5.0):
    """Oracle O1 (the direct line-integral FBP in C, FP64, OpenMP over all the
    host's threads) on a bounded sample: the row filter of all projections
    (numpy), then z slices spread over the volume for `budget_s` seconds,
    scaled to all nz slices."""
    from oracle import direct, filters
    from oracle.geometry import Geometry

    g = Geometry(nz=NZ, n=N, n_theta=NT, h=H, w=W, phi=TILT)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    fd = direct.filter_rows(data_np, g, filters.SHEPP_LOGAN)
    t_filter = time.perf_counter() - t0
    t_slices, done = 0.0, 0
    for k in range(NZ):
        z = (k * 97) % NZ
        t1 = time.perf_counter()
        direct.adjoint(fd, g, z_range=(z, z + 1))
        t_slices += time.perf_counter() - t1
        done += 1
        if t_slices >= budget_s:
            break
    t_total = t_filter + t_slices / done * NZ
    return {"value": round(NZ * N * N / t_total / 1e9, 9), "unit": "GVoxel/s", "cores": threads,
            "kind": "oracle",
            "sample": f"O1 direct bilinear FBP (C, FP64, OpenMP): row filter of all {NT} projections "
                      f"and {done} of {NZ} z slices, scaled linearly ({t_filter + t_slices:.1f} s "
                      f"measured, {t_total:.0f} s extrapolated)"}


SERVE_CLASSES = [(128, 128, 180), (256, 256, 400), (256, 512, 720)]  # (nz, n, n_theta)
SERVE_TILTS = (20.0, 25.0, 30.0, 35.0, 40.0)


def serving_classes(dev, host=False):
    """Per class and tilt: 30 seeded ellipsoids projected at that tilt with
    0.5% noise (detector nz x n); pinned host memory with host=True."""
    classes = []
    for (nz, n, nt), seed in zip(SERVE_CLASSES, (10, 11, 12)):
        h, w = nz, n
        ells = synth.random_ellipsoids(30, nz, n, seed=seed)
        per_tilt = {}
        for deg in SERVE_TILTS:
            d = synth.project_ellipsoids(ells, nt, h, w, np.deg2rad(deg), device=dev, dtype=torch.float32)
            d = synth.add_noise(d, 0.005, seed=seed + 100).contiguous()
            per_tilt[deg] = d.cpu().pin_memory() if host else d
        classes.append((nz, n, nt, h, w, per_tilt))
    return classes


def serving(dev, classes, count, rate=20.0, host=False, seed=0):
    """Poisson stream of fp16-gridded FBP requests over the three size classes
    and the tilt set; host=True: data in pinned host memory and every volume
    returned to pinned host memory (latency from arrival to the result on the
    host)."""
    from paper_2401_11101_amd.serve import Server, run_poisson

    srv = Server(max_slots=4, hbm_budget=32 << 30, storage_dtype="f16", data_dtype="f32", device=dev,
                 result_on_host=host, keep_results=False)
    # warm every class once (plans, slots, kernels), then the timed stream
    run_poisson(srv, classes, rate=1000.0, count=6, seed=99)
    srv.finished.clear()
    st = run_poisson(srv, classes, rate=rate, count=count, seed=seed)
    srv.close()
    return {"requests": st["requests"], "rate_per_s": rate, "p50_ms": round(st["p50_ms"], 3),
            "p99_ms": round(st["p99_ms"], 3), "mean_ms": round(st["mean_ms"], 3),
            "throughput_rps": round(st["throughput_rps"], 3), "gvoxel_per_s": round(st["gvoxel_per_s"], 4),
            "classes": "U{128^3/180, 256^3/400, 512x512x256/720}, each request's data projected at "
                       "its own tilt, tilts U{20,25,30,35,40} deg, fp16 storage, 4 slots, " +
                       ("data in pinned host memory, volumes returned to pinned host memory"
                        if host else "data resident on the device")}


def serving_sweep(dev, classes, rates=(50.0, 100.0, 200.0, 400.0, 800.0), count=300):
    """Arrival-rate sweep up to saturation: throughput and latency per rate."""
    rows = []
    for k, rate in enumerate(rates):
        r = serving(dev, classes, count, rate=rate, seed=10 + k)
        rows.append({key: r[key] for key in ("rate_per_s", "requests", "throughput_rps", "p50_ms",
                                             "p99_ms", "gvoxel_per_s")})
    return rows


def large_volume(dev, steps):
    """1024 x 1024 x 512 volume, 1500 projections 512 x 1024, tilt 20 deg, fp16 data
    and storage, x3 output in z-chunks of 64."""
    from paper_2401_11101_amd import Plan

    nz, n, nt, h, w = 512, 1024, 1500, 512, 1024
    ells = synth.random_ellipsoids(20, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, np.deg2rad(20.0), device=dev, dtype=torch.float32,
                                 theta_chunk=8)
    d = synth.apply_speckle(d, 0.1, seed=1).half().contiguous()
    plan = Plan(nz, n, nt, h, w, np.deg2rad(20.0), data_dtype="f16", storage_dtype="f16", z_chunk=64)
    vol = torch.empty((nz, n, n), dtype=torch.float32, device=dev)
    ms, _, st = time_op(lambda: plan.fbp(d, out=vol), steps, 1, torch.cuda.current_stream(), plan)
    # data and volume in pinned host memory: projections stream in, z-chunks
    # of 64 slices stream out through the device staging buffers
    hd = d.cpu().pin_memory()
    hv = torch.empty((nz, n, n), dtype=torch.float32, pin_memory=True)
    ms_host = _event_ms(lambda: plan.fbp_host(hd, out=hv), 2, torch.cuda.current_stream())
    same = bool(torch.equal(hv, vol.cpu()))
    return {"workload": "FBP 1024x1024x512 from 1500 projections 512x1024, tilt 20 deg, fp16 data "
                        "and storage, z-chunks of 64", "ms_per_step": round(ms, 3),
            "gvoxel_per_s": round(nz * n * n / (ms * 1e-3) / 1e9, 4),
            "stages_ms_per_step": {k: round(v[0] / steps, 3) for k, v in st.items()},
            "workspace_gb": round(plan.work.numel() / 2**30, 3),
            "host_io": {"ms": round(ms_host, 3), "gvoxel_per_s": round(nz * n * n / (ms_host * 1e-3) / 1e9, 4),
                        "equal_to_device_run": same,
                        "note": "lamino_fbp_host: fp16 projections from pinned host memory (read twice: "
                                "input scan, transforms), volume to pinned host memory in z-chunks of 64"}}


def cg_reconstruction(dev, iters=20):
    """CGLS, 20 iterations: 256^3 volume, 720 projections 256 x 320, tilt 30 deg, bf16 storage."""
    from paper_2401_11101_amd import Plan
    from paper_2401_11101_amd.autograd import cgls

    nz = n = h = 256
    w, nt = 320, 720
    ells = synth.random_ellipsoids(50, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, np.deg2rad(30.0), device=dev, dtype=torch.float32)
    plan = Plan(nz, n, nt, h, w, np.deg2rad(30.0), storage_dtype="bf16")
    res = []
    cgls(plan, d, iters=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cgls(plan, d, iters=iters, callback=lambda k, x, r: res.append(r))
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    return {"workload": "CGLS 20 iterations, 256^3 volume, 720 projections 256x320, tilt 30 deg, "
                        "bf16 storage", "seconds": round(t, 3), "ms_per_iteration": round(t * 1e3 / iters, 3),
            "residual_first_last": [round(res[0], 4), round(res[-1], 4)]}


def _event_ms(fn, reps, stream):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def admm_tv_reconstruction(dev, outer=4, inner=4):
    """TV-regularised ADMM (Appendix A), 256^3 volume, 720 projections 256 x 320,
    tilt 30 deg, bf16 storage; plus each TV kernel against the HBM roofline."""
    from paper_2401_11101_amd import Plan, tv

    nz = n = h = 256
    w, nt = 320, 720
    ells = synth.random_ellipsoids(50, nz, n, seed=0)
    d = synth.project_ellipsoids(ells, nt, h, w, np.deg2rad(30.0), device=dev, dtype=torch.float64)
    d = synth.add_noise(d, 0.01, seed=1).float().contiguous()
    plan = Plan(nz, n, nt, h, w, np.deg2rad(30.0), storage_dtype="bf16")
    stream = torch.cuda.current_stream()
    # threshold alpha / rho = 0.1 against edge gradients of O(0.1-1) in density units
    alpha, rho = 0.1, 1.0
    vol = torch.zeros(plan.shape_vol, dtype=torch.float32, device=dev)
    st = tv.AdmmTV(plan, alpha, rho)
    st.run(d, vol, 1, 1, resume=False)  # warm-up (kernels, state)
    vol.zero_()
    torch.cuda.synchronize()
    plan.stage_times(reset=True)
    plan.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    st.run(d, vol, outer, inner, resume=False)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    plan.profile(False)
    op_ms = sum(v[0] for v in plan.stage_times(reset=True).values())
    r = plan.fwd(vol) - d
    gv = tv.grad(vol)
    tvn = float(torch.sqrt((gv.double() ** 2).sum(0)).sum())
    obj = 0.5 * float((r.double() ** 2).sum()) + alpha * tvn
    psi = st.shift.double() + st.lam.double() / rho
    zero = float((psi.abs().sum(0) == 0).double().mean())
    gmag = torch.sqrt((gv.double() ** 2).sum(0)).flatten()
    gq = [float(x) for x in torch.quantile(gmag[:: max(1, gmag.numel() // 1000000)],
                                           torch.tensor([0.5, 0.9, 0.99], dtype=torch.float64,
                                                        device=dev))]
    # the TV kernels on their own (algorithmic bytes per voxel: reads + writes)
    nv = nz * n * n
    mu = torch.randn(plan.shape_vol, device=dev)
    lam = torch.randn((3,) + plan.shape_vol, device=dev) * 0.1
    shift = torch.zeros_like(lam)
    base = torch.randn_like(mu)
    out = torch.empty_like(mu)
    g3 = torch.empty_like(lam)
    kernels = {
        "k_tv_grad": (lambda: tv.grad(mu, out=g3), 16),
        "k_tv_term": (lambda: tv.tv_term(mu, rho, shift=shift, base=base, out=out), 24),
        "k_tv_shrink": (lambda: tv.shrink(mu, lam, shift, alpha, rho), 40),
        "k_tv_div": (lambda: tv.div(lam, out=out), 16),
    }
    krep = {}
    for name, (fn, bpv) in kernels.items():
        kms = _event_ms(fn, 20, stream)
        gbs = bpv * nv / (kms * 1e-3) / 1e9
        krep[name] = {"ms": round(kms, 4), "bytes_per_voxel": bpv, "achieved_GBs": round(gbs, 1),
                      "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return {"workload": f"TV-ADMM {outer} outer x {inner} CG iterations, 256^3 volume, 720 projections "
                        "256x320, tilt 30 deg, bf16 storage, 50 ellipsoids + 1% noise",
            "alpha": alpha, "rho": rho, "ms_total": round(ms, 3),
            "ms_per_outer_iteration": round(ms / outer, 3),
            "operator_ms": round(op_ms, 3), "tv_and_cg_ms": round(ms - op_ms, 3),
            "operator_applications": 2 + 2 * outer * inner,
            "objective": obj, "psi_zero_fraction": round(zero, 4),
            "grad_magnitude_p50_p90_p99": [round(x, 4) for x in gq],
            "tv_kernels": krep}


def table1(dev, sizes=(256, 512, 1024, 1536, 2048)):
    """The paper's timing-table workload: N projections of N x N, 8-bit data,
    tilt 20 deg, N^3 volume (float32).  Fourier-route FBP (fp32 and fp16
    storage) against the direct line-integral FBP, device-resident, one timed
    run each after a warm-up; plus a PCIe-inclusive run at N = 1024."""
    from paper_2401_11101_amd import Plan

    tilt = np.deg2rad(20.0)
    stream = torch.cuda.current_stream()
    rows = []
    e2e = None
    for N in sizes:
        log(f"table1: N = {N}")
        ells = synth.random_ellipsoids(20, N, N, seed=0)
        d = synth.project_ellipsoids(ells, N, N, N, tilt, device=dev, dtype=torch.float32, theta_chunk=8)
        d8 = torch.clamp(d * (255.0 / float(d.max())), 0, 255).round().to(torch.uint8)
        del d
        torch.cuda.empty_cache()
        vol = torch.empty((N, N, N), dtype=torch.float32, device=dev)
        row = {"N": N}
        # float32 storage needs ~2x the fp16 workspace: when it does not fit
        # beside the data and the volume, the slab planes go to host memory
        try:
            plan = Plan(N, N, N, N, N, tilt, data_dtype="u8", storage_dtype="f32")
            row["fourier_f32_layout"] = "device"
        except torch.cuda.OutOfMemoryError:
            torch.cuda.empty_cache()
            plan = Plan(N, N, N, N, N, tilt, data_dtype="u8", storage_dtype="f32", hbm_budget=150 << 30)
            row["fourier_f32_layout"] = (f"out of core: spectra {'host' if plan.info.spill_spectra else 'device'}, "
                                         f"slab planes {'host' if plan.info.spill_slabs else 'device'} "
                                         f"({plan.info.host_bytes / 2**30:.1f} GiB pinned host memory)")
        row["fourier_f32_ms"] = round(_event_ms(lambda: plan.fbp(d8, out=vol), 1, stream), 3)
        del plan
        torch.cuda.empty_cache()
        # the direct FBP needs only the plan's tables: it runs on the fp16 plan
        plan = Plan(N, N, N, N, N, tilt, data_dtype="u8", storage_dtype="f16")
        row["fourier_f16_ms"] = round(_event_ms(lambda: plan.fbp(d8, out=vol), 1, stream), 3)
        if N == 1024:
            e2e = _end_to_end(plan, d8, vol, stream)
        row["direct_ms"] = round(_event_ms(lambda: plan.direct_fbp(d8, out=vol), 1, stream), 3)
        row["direct_voxel_angles_per_s"] = float(f"{float(N) ** 4 / (row['direct_ms'] * 1e-3):.4g}")
        del plan, vol, d8
        torch.cuda.empty_cache()
        for storage in ("f32", "f16"):
            if f"fourier_{storage}_ms" in row:
                row[f"gain_{storage}"] = round(row["direct_ms"] / row[f"fourier_{storage}_ms"], 3)
        row["fourier_f16_gvoxel_per_s"] = round(N ** 3 / (row["fourier_f16_ms"] * 1e-3) / 1e9, 4)
        rows.append(row)
    return {"workload": "N projections of N x N over [0, 2pi), 8-bit data, tilt 20 deg, N^3 float32 "
                        "volume, Shepp-Logan; device-resident, one run after a warm-up",
            "rows": rows, "end_to_end_N1024_f16": e2e,
            "paper_context": "A100 40 GB, times including the chunked host-device pipeline: Fourier "
                             "3.0 / 8.6 / 21.1 s and direct 9.3 / 52.1 / 222.1 s at N = 1024 / 1536 / 2048"}


def _u8_projections(N, tilt, dev, chunk=8):
    """8-bit ellipsoid projections of the N-cube workload, generated a few
    angles at a time (the float32 set of N = 3072 alone would take 116 GB)."""
    ells = synth.random_ellipsoids(20, N, N, seed=0)
    theta = synth.angles(N)
    probe = synth.project_ellipsoids(ells, 32, N, N, tilt, theta=theta[::max(1, N // 32)][:32], device=dev,
                                     dtype=torch.float32, theta_chunk=chunk)
    scale = 255.0 / (1.1 * float(probe.max()))
    del probe
    d8 = torch.empty((N, N, N), dtype=torch.uint8, device=dev)
    for t0 in range(0, N, chunk):
        t1 = min(N, t0 + chunk)
        d = synth.project_ellipsoids(ells, t1 - t0, N, N, tilt, theta=theta[t0:t1], device=dev,
                                     dtype=torch.float32, theta_chunk=chunk)
        d8[t0:t1] = torch.clamp(d * scale, 0, 255).round().to(torch.uint8)
        if t0 % (64 * chunk) == 0:
            log(f"  projections {t1} / {N}")
    return d8


def table1_3072(dev):
    """The N = 3072 row of the timing table: 3072 projections of 3072 x 3072,
    8-bit data, tilt 20 deg, 3072^3 float32 volume (116 GB).  fp16 storage;
    the detector is padded to the next power of two (4096, pad factor 1.33)
    instead of 2x (8192, whose spectra alone would take 412 GB); the slab
    planes live in pinned host memory when the device cannot hold them beside
    the volume, the data and the spectra.  One timed run each of the Fourier
    and the direct FBP, data and volume resident on the device."""
    from paper_2401_11101_amd import Plan

    N = 3072
    tilt = np.deg2rad(20.0)
    torch.cuda.empty_cache()
    torch._C._host_emptyCache()  # pinned blocks cached from earlier rows
    # the plan first: its device workspace takes what the volume and the data
    # leave, and its pinned host buffer may be refused by the host
    budget = torch.cuda.mem_get_info()[0] - 5 * N ** 3 - (10 << 30)
    log(f"table1: N = 3072 (plan, {budget / 2**30:.0f} GiB of device memory for the workspace)")
    try:
        plan = Plan(N, N, N, N, N, tilt, data_dtype="u8", storage_dtype="f16", pad_u=1.0, pad_v=1.0,
                    hbm_budget=budget)
    except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
        torch.cuda.empty_cache()
        return {"N": N, "not_run": f"plan allocation failed: {str(e).splitlines()[0]}",
                "device_budget_gib": round(budget / 2**30, 1)}
    i = plan.info
    log("table1: N = 3072 (data)")
    d8 = _u8_projections(N, tilt, dev)
    vol = torch.empty((N, N, N), dtype=torch.float32, device=dev)
    row = {"N": N, "pad": [1.0, 1.0], "w_p": i.w_p, "h_p": i.h_p, "grid": i.grid,
           "fourier_f16_layout": (f"spectra {'host' if i.spill_spectra else 'device'}, slab planes "
                                  f"{'host' if i.spill_slabs else 'device'} ({i.host_bytes / 2**30:.1f} GiB "
                                  f"pinned host memory), device workspace {i.work_bytes / 2**30:.1f} GiB")}
    log("table1: N = 3072 (Fourier FBP)")
    plan.fbp(d8, out=vol)  # warm-up: binds the host buffer, uploads the tables
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.fbp(d8, out=vol)
    torch.cuda.synchronize()
    row["fourier_f16_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    row["fourier_f16_gvoxel_per_s"] = round(N ** 3 / (row["fourier_f16_ms"] * 1e-3) / 1e9, 4)
    row["finite"] = bool(torch.isfinite(vol[::256]).all())
    # the direct FBP uses the plan's tables only: its filtered rows (116 GB)
    # take the place of the Fourier workspace
    plan.work = None
    torch.cuda.empty_cache()
    log("table1: N = 3072 (direct FBP)")
    t0 = time.perf_counter()
    plan.direct_fbp(d8, out=vol)
    torch.cuda.synchronize()
    row["direct_ms"] = round((time.perf_counter() - t0) * 1e3, 1)
    row["direct_voxel_angles_per_s"] = float(f"{float(N) ** 4 / (row['direct_ms'] * 1e-3):.4g}")
    row["gain_f16"] = round(row["direct_ms"] / row["fourier_f16_ms"], 3)
    del plan, vol, d8
    torch.cuda.empty_cache()
    row["paper_context"] = "A100 40 GB, including the host pipeline: Fourier 77.7 s, direct 1002.2 s"
    return row


def _end_to_end(plan, d8, vol, stream):
    """Pinned-host 8-bit data -> device, FBP, volume -> pinned host, one run."""
    h_in = torch.empty(d8.shape, dtype=torch.uint8, pin_memory=True)
    h_in.copy_(d8.cpu())
    h_out = torch.empty(vol.shape, dtype=torch.float32, pin_memory=True)
    dd = torch.empty_like(d8)

    def run():
        dd.copy_(h_in, non_blocking=True)
        plan.fbp(dd, out=vol)
        h_out.copy_(vol, non_blocking=True)

    ms = _event_ms(run, 1, stream)
    N = vol.shape[0]
    return {"ms": round(ms, 3), "gvoxel_per_s": round(N ** 3 / (ms * 1e-3) / 1e9, 4),
            "bytes_h2d": d8.numel(), "bytes_d2h": vol.numel() * 4}


def search_sweeps(dev, data):
    """Axis sweep (41 offsets, -10 .. 10 columns in steps of 0.5) and tilt sweep
    (21 tilts, 23 .. 27 deg in steps of 0.2) of one slice of the 256^3 workload."""
    from paper_2401_11101_amd import Plan, search

    stream = torch.cuda.current_stream()
    plan = Plan(NZ, N, NT, H, W, TILT)
    shifts = [0.5 * k for k in range(-20, 21)]
    search.center_sweep(plan, data, shifts[:2], z=NZ // 2)
    ms_c = _event_ms(lambda: search.center_sweep(plan, data, shifts, z=NZ // 2), 1, stream)
    del plan
    tilts = np.deg2rad(23.0 + 0.2 * np.arange(21))
    t0 = time.perf_counter()
    search.tilt_sweep(NZ, N, NT, H, W, tilts, data, z=NZ // 2)
    torch.cuda.synchronize()
    ms_t = (time.perf_counter() - t0) * 1e3
    return {"workload": "one slice (z = nz/2) of the 256^3 / 400-projection FBP per candidate",
            "center_sweep": {"candidates": len(shifts), "ms": round(ms_c, 2),
                             "ms_per_slice": round(ms_c / len(shifts), 3)},
            "tilt_sweep": {"candidates": len(tilts), "ms_wall": round(ms_t, 2),
                           "ms_per_slice": round(ms_t / len(tilts), 3),
                           "note": "includes the FP64 host tables and their upload for every tilt"}}


def copy_calibration(nbytes=1 << 30):
    """Plain copies of `nbytes` with 4-, 8- and 16-byte lane accesses (and the
    runtime's own device copy), each once: under rocprofv3 --pmc their
    FETCH_SIZE / WRITE_SIZE give the counters' scale for known traffic."""
    import ctypes

    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2401_11101_amd", "lib", "libcopycalib.so"))
    lib.lamino_calib_copy.restype = ctypes.c_int
    lib.lamino_calib_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_int, ctypes.c_void_p]
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    s = torch.cuda.current_stream()
    for width in (4, 8, 16):
        rc = lib.lamino_calib_copy(x.data_ptr(), y.data_ptr(), nbytes, width, s.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"lamino_calib_copy width {width}: {rc}")
    y.copy_(x)
    torch.cuda.synchronize()
    assert bool((y == 1).all())
    print(json.dumps({"copy_bytes_each_way": nbytes, "widths": [4, 8, 16, "runtime"]}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the serving stream (0 skips it)")
    ap.add_argument("--no-serve-host", action="store_true",
                    help="skip the serving stream with data and results in pinned host memory")
    ap.add_argument("--extra", action="store_true",
                    help="also time the 1024^2 x 512 volume, CGLS and the TV-regularised ADMM")
    ap.add_argument("--admm", action="store_true",
                    help="also time the TV-regularised ADMM and its kernels (part of --extra)")
    ap.add_argument("--large", action="store_true",
                    help="also time the 1024^2 x 512 volume (part of --extra)")
    ap.add_argument("--table1-3072", action="store_true",
                    help="the N = 3072 row of the timing table (fp16, ~2 minutes, 116 GB volume)")
    ap.add_argument("--table1", action="store_true",
                    help="also run the Fourier-vs-direct timing table (N = 256 .. 2048, 8-bit data)")
    ap.add_argument("--search", action="store_true",
                    help="also time the rotation-axis and tilt sweeps (one slice per candidate)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 1 GiB device copies (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the operators would shard over angles, frequency slabs and volume columns "
              "with two all-to-all exchanges; only the one-GPU share is built)", file=sys.stderr)
        sys.exit(2)
    from paper_2401_11101_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    log(f"generating the 256^3 / 400-projection data on {torch.cuda.get_device_name(dev)}")
    data = make_data(dev)
    data16 = data.half()
    p32 = Plan(NZ, N, NT, H, W, TILT)
    p16 = Plan(NZ, N, NT, H, W, TILT, data_dtype="f16", storage_dtype="f16")
    vol32 = torch.empty((NZ, N, N), dtype=torch.float32, device=dev)
    vol16 = torch.empty_like(vol32)
    log("timing fp32 FBP")
    ms32, wall32, st32 = time_op(lambda: p32.fbp(data, out=vol32), args.steps, args.warmup, stream, p32)
    log("timing fp16-storage FBP")
    ms16, wall16, st16 = time_op(lambda: p16.fbp(data16, out=vol16), args.steps, args.warmup, stream, p16)
    e16 = float((vol16 - vol32).norm() / vol32.norm())
    # the two volumes, kept for the accuracy check of the CPU leg
    v32_host, v16_host = vol32.cpu().numpy(), vol16.cpu().numpy()
    # Fourier-route FBP against the direct (bilinear line-integral) FBP on the
    # same data: a property of the two discretisations (both GPU paths match
    # their FP64 definitions in the tests)
    vdir = p32.direct_fbp(data)
    gap_direct = float((vol32.double() - vdir.double()).norm() / vdir.double().norm())
    del vdir
    log("timing fp32 forward and adjoint")
    dfwd = torch.empty_like(data)
    ms_fwd, _, st_fwd = time_op(lambda: p32.fwd(vol32, out=dfwd), max(3, args.steps // 2), 1, stream, p32)
    ms_adj, _, _ = time_op(lambda: p32.adj(data, out=vol32), max(3, args.steps // 2), 1, stream)
    log("timing the FBP of 16-bit raw counts (dark/flat + -log fused into the first kernel)")
    raw, dark, flat = synth.raw_counts(0.02 * data.double().cpu().numpy(), seed=3)
    raw_d = torch.from_numpy(raw).to(dev)
    dark_d, flat_d = torch.from_numpy(dark).to(dev), torch.from_numpy(flat).to(dev)
    praw = Plan(NZ, N, NT, H, W, TILT, data_dtype="u16")
    ms_raw, _, st_raw = time_op(lambda: praw.fbp_raw(raw_d, dark_d, flat_d, out=vol32),
                                max(3, args.steps // 2), 1, stream, praw)
    del praw
    vox = NZ * N * N
    work = algorithmic_work(p32.info, 8, 4)
    line = {
        "metric": "GVoxel/s FBP fp32 vs fp16-gridded at stated rel-L2 err; p50/p99 request latency",
        "value": round(vox / (ms32 * 1e-3) / 1e9, 4),
        "unit": "GVoxel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": ("float32 data, spectra, slab planes and accumulation, FP64 tables; the gridding and "
                       "x3 products run on the matrix cores as three bf16 products per term (hi hi, hi lo, "
                       "lo hi of bf16 hi / lo splits, ~2^-17 relative per term)"),
        "data": "synthetic",
        "config": {"workload": "FBP of a 256x256x256 volume from 400 projections over [0, 2pi), "
                               "tilt 25 deg, detector 256x256, 50 ellipsoids + 0.5% noise, Shepp-Logan",
                   "parallelism": "none (1 GPU)"},
        "rel_l2": {"f32_vs_exact_fourier_fbp": None, "f16_vs_exact_fourier_fbp": None,
                   "required": {"f32": 1e-4, "f16": 1e-2},
                   "f16_vs_f32": round(e16, 6),
                   "fourier_vs_direct_fbp": round(gap_direct, 5)},
        "fp16_gridded": {"value": round(vox / (ms16 * 1e-3) / 1e9, 4), "ms_per_step": round(ms16, 4),
                         "speedup_vs_f32": round(ms32 / ms16, 3)},
        "operators_ms": {"fwd_f32": round(ms_fwd, 4), "adj_f32": round(ms_adj, 4)},
        "fbp_raw_u16": {"ms_per_step": round(ms_raw, 4),
                        "detector_stage_ms": round(st_raw["detector"][0] / max(3, args.steps // 2), 4),
                        "note": "16-bit counts, dark/flat correction and -log inside the first "
                                "detector kernel, fp32 storage"},
        "stages_ms_per_step": {
            "f32": {k: round(v[0] / args.steps, 4) for k, v in st32.items()},
            "f16": {k: round(v[0] / args.steps, 4) for k, v in st16.items()},
            "fwd_f32": {k: round(v[0] / max(3, args.steps // 2), 4) for k, v in st_fwd.items()},
        },
        "wall_ms_per_step": {"f32": round(wall32, 4), "f16": round(wall16, 4)},
        "roofline": roofline(st32, work, args.steps, p32.info),
    }
    if args.serve_requests:
        classes = serving_classes(dev)
        log(f"serving: {args.serve_requests} Poisson requests at 20/s")
        line["serving"] = serving(dev, classes, args.serve_requests)
        log("serving: arrival-rate sweep")
        line["serving_sweep"] = serving_sweep(dev, classes)
        del classes
        if not args.no_serve_host:
            log(f"serving from host memory: {args.serve_requests} Poisson requests at 20/s")
            line["serving_host"] = serving(dev, serving_classes(dev, host=True), args.serve_requests,
                                           host=True)
    if args.extra or args.large:
        log("timing the 1024^2 x 512 volume")
        line["large_volume"] = large_volume(dev, 3)
    if args.extra:
        log("timing CGLS")
        line["cgls"] = cg_reconstruction(dev)
    if args.extra or args.admm:
        log("timing the TV-regularised ADMM")
        line["admm_tv"] = admm_tv_reconstruction(dev)
    if args.table1:
        line["table1"] = table1(dev)
    if args.table1_3072:
        try:
            line["table1_3072"] = table1_3072(dev)
        except (RuntimeError, torch.cuda.OutOfMemoryError) as e:
            line["table1_3072"] = {"N": 3072, "not_run": str(e).splitlines()[0]}
    if args.search or args.extra:
        log("timing the axis and tilt sweeps")
        line["search"] = search_sweeps(dev, data)
    if not args.no_cpu:
        log("timing the CPU oracle baseline (bounded sample)")
        base, acc = cpu_baseline(data.double().cpu().numpy(), {"f32": v32_host, "f16": v16_host})
        line["cpu_baseline"] = base
        line["rel_l2"]["f32_vs_exact_fourier_fbp"] = round(acc["rel_l2"]["f32"], 9)
        line["rel_l2"]["f16_vs_exact_fourier_fbp"] = round(acc["rel_l2"]["f16"], 7)
        line["rel_l2"]["sampled_columns"] = acc["columns"]
        line["rel_l2"]["note"] = ("exact FP64 Fourier FBP sums of the sampled columns (all z) on the "
                                  "float32 data; the fp16 path also rounds its input to float16")
        log("timing the CPU direct-FBP oracle (bounded sample)")
        line["cpu_direct_fbp"] = cpu_direct_fbp(data.double().cpu().numpy())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
