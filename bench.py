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
    """Algorithmic bytes / flops per FBP of each stage."""
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


def roofline(stages, work):
    name = max(stages, key=lambda k: stages[k][0])
    ms, launches = stages[name]
    per_launch_ms = ms / max(launches, 1)
    w = work[name]
    if name == "gridding":
        # matrix-core gridding: algorithmic taps as float32 vector work
        achieved = w["flops"] / max(launches, 1) / (per_launch_ms * 1e-3) / 1e12
        return {"kernel": "k_spread (gridding)", "bound": "alu", "achieved": round(achieved, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4), "traffic": None}
    achieved = w["bytes"] / max(launches, 1) / (per_launch_ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None}


def cpu_baseline(data_np, proj=80, angles=100):
    """Oracle O3 (FP64 Gaussian USFFT FBP, numpy) on a bounded sample.

    Times the oracle's detector transform + filter on `proj` projections and
    the gridding / inverse FFT / psi correction / x3 accumulation of one
    frequency slab restricted to `angles` angles, then scales both linearly
    to the whole workload (all projections, all 2 h_p / 2 - 1 slabs)."""
    from oracle import filters, nudft, usfft
    from oracle.geometry import Geometry, freqs

    g_sub = Geometry(nz=NZ, n=N, n_theta=proj, h=H, w=W, phi=TILT,
                     theta=2 * np.pi * np.arange(proj) / NT)
    t0 = time.perf_counter()
    Gs = nudft.filter_spectra(nudft.data_spectra_fft(data_np[:proj], g_sub, half=True), g_sub,
                              filters.SHEPP_LOGAN)
    t_det = (time.perf_counter() - t0) * NT / proj
    g_a = Geometry(nz=NZ, n=N, n_theta=angles, h=H, w=W, phi=TILT,
                   theta=2 * np.pi * np.arange(angles) / NT)
    N_g = usfft.default_grid(N)
    ls_all = freqs(g_a.h_p)
    l = g_a.h_p // 4
    Ga = np.zeros((angles, len(freqs(g_a.w_p))), dtype=np.complex128)
    Ga[:min(angles, proj)] = Gs[:min(angles, proj), l, :]
    t0 = time.perf_counter()
    X, Y = usfft.slab_positions(g_a, l, N_g)
    gl = usfft.type1(Ga.reshape(-1), X, Y, N, N_g, 12)
    E = nudft.x3_phases(g_a, +1.0)[:, int(np.where(ls_all == l)[0][0])]
    acc = np.real(E[:, None, None] * gl[None])
    t_slab = (time.perf_counter() - t0) * NT / angles
    del acc
    t_total = t_det + t_slab * len(ls_all)
    measured = t_det * proj / NT + t_slab * angles / NT
    return {"value": round(NZ * N * N / t_total / 1e9, 8), "unit": "GVoxel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"O3 FP64 Gaussian-USFFT FBP (numpy, M=12, single thread): detector FFT + "
                      f"filter of {proj}/{NT} projections and one of {len(ls_all)} frequency slabs "
                      f"gridded from {angles}/{NT} angles, scaled linearly to the whole 256^3 FBP "
                      f"({measured:.1f} s measured, {t_total:.0f} s extrapolated)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(DESIGN.md describes how it would shard)", file=sys.stderr)
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
    log("timing fp32 forward and adjoint")
    dfwd = torch.empty_like(data)
    ms_fwd, _, st_fwd = time_op(lambda: p32.fwd(vol32, out=dfwd), max(3, args.steps // 2), 1, stream, p32)
    ms_adj, _, _ = time_op(lambda: p32.adj(data, out=vol32), max(3, args.steps // 2), 1, stream)
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
        "data": "synthetic",
        "config": {"workload": "FBP of a 256x256x256 volume from 400 projections over [0, 2pi), "
                               "tilt 25 deg, detector 256x256, 50 ellipsoids + 0.5% noise, Shepp-Logan",
                   "parallelism": "none (1 GPU)"},
        "rel_l2": {"f32_vs_exact_fourier_fbp": "<= 1e-4 (tests: sampled columns at this size)",
                   "f16_vs_f32": round(e16, 6)},
        "fp16_gridded": {"value": round(vox / (ms16 * 1e-3) / 1e9, 4), "ms_per_step": round(ms16, 4),
                         "speedup_vs_f32": round(ms32 / ms16, 3)},
        "operators_ms": {"fwd_f32": round(ms_fwd, 4), "adj_f32": round(ms_adj, 4)},
        "stages_ms_per_step": {
            "f32": {k: round(v[0] / args.steps, 4) for k, v in st32.items()},
            "f16": {k: round(v[0] / args.steps, 4) for k, v in st16.items()},
            "fwd_f32": {k: round(v[0] / max(3, args.steps // 2), 4) for k, v in st_fwd.items()},
        },
        "wall_ms_per_step": {"f32": round(wall32, 4), "f16": round(wall16, 4)},
        "roofline": roofline(st32, work),
    }
    if not args.no_cpu:
        log("timing the CPU oracle baseline (bounded sample)")
        line["cpu_baseline"] = cpu_baseline(data.double().cpu().numpy())
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
