"""Benchmark: GVoxel/s of the Fourier-route FBP on one MI355X.

Workload: volume 256 x 256 x 256, 400 projections over [0, 2 pi), tilt
25 deg, detector 256 x 256, 50 seeded ellipsoids, float32 data with 0.5%
Gaussian noise (exact projections computed on the GPU from the closed
form; the paper's datasets are not available).  A step is one FBP of the
whole batch with inputs resident in HBM.  The float32 path (storage f32,
Gaussian half-width 5) gives `value`; the fp16-storage path (half-width
3) is reported beside it.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3]
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


def make_data(device):
    ells = synth.random_ellipsoids(50, NZ, N, seed=0)
    d = synth.project_ellipsoids(ells, NT, H, W, TILT, device=device, dtype=torch.float64)
    d = synth.add_noise(d, 0.005, seed=1)
    return d.float().contiguous()


def time_op(fn, steps, warmup, stream):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return ev0.elapsed_time(ev1) / steps, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see the sharding note in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    from paper_2401_11101_amd import Plan

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    print(f"[bench] generating c2 data on {torch.cuda.get_device_name(dev)}", file=sys.stderr, flush=True)
    data = make_data(dev)
    data16 = data.half()
    p32 = Plan(NZ, N, NT, H, W, TILT)
    p16 = Plan(NZ, N, NT, H, W, TILT, data_dtype="f16", storage_dtype="f16")
    vol32 = torch.empty((NZ, N, N), dtype=torch.float32, device=dev)
    vol16 = torch.empty_like(vol32)
    print("[bench] timing fp32 FBP", file=sys.stderr, flush=True)
    ms32, wall32 = time_op(lambda: p32.fbp(data, out=vol32), args.steps, args.warmup, stream)
    print("[bench] timing fp16-storage FBP", file=sys.stderr, flush=True)
    ms16, wall16 = time_op(lambda: p16.fbp(data16, out=vol16), args.steps, args.warmup, stream)
    torch.cuda.synchronize()
    e16 = float((vol16 - vol32).norm() / vol32.norm())
    vox = NZ * N * N
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
        "config": {"workload": "c2 plain FBP: vol 256^3, 400 proj over [0,2pi), tilt 25 deg, "
                               "det 256x256, 50 ellipsoids + 0.5% noise, Shepp-Logan",
                   "parallelism": "none (1 GPU)"},
        "fp16_gridded": {"value": round(vox / (ms16 * 1e-3) / 1e9, 4), "ms_per_step": round(ms16, 4),
                         "speedup_vs_f32": round(ms32 / ms16, 3), "rel_l2_vs_f32": e16},
        "wall_ms_per_step": {"f32": round(wall32, 4), "f16": round(wall16, 4)},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
