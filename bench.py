"""Benchmark of the SDE-ensemble hot path on one MI355X.

Default workload: the Josephson-junction (f, D) scan -- 128 x 128 points
(f = 0.5 i/127, D = 10^(-4 + 3 j/127)), 1024 paths per point, 2*10^5
stochastic-Heun steps of dt = 2 pi/omega/200 (10^5 transient), FP32 state
with FP64 <v> accumulation, all 16384 points in one persistent launch.
A "step" of this benchmark is one such full integration (3.36e12
path-steps); inputs (parameters) are resident before timing starts.

Prints one JSON line with the throughput in path-steps/s, the ALU roofline
fraction of the integration kernel and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import sde_inputs  # noqa: E402

# ---------------------------------------------------------------------------
# ALU roofline of the Josephson-junction kernel.
# Peak: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 full-rate VALU lane
# slots per second (a wave64 VALU instruction occupies its SIMD for 4 cycles;
# packed FP32 forms are not used).  Algorithmic cost of one Heun path-step of
# Eq. 1, counted from the method (not from the compiled code), each operation
# weighted by its issue cost in full-rate slots:
#   Philox4x32-10 / 4 steps: 20 wide 32x32->64 multiplies, 40 xor
#   Box-Muller / 2 steps:    2 shifts, 1 add, 2 int->float, 2 scale,
#                            1 log2, 1 mul, 1 sqrt, 1 sin, 1 cos, 2 mul
#   Heun step (Alg. 2):      2 sin + 13 add/mul/fma (drift twice, predictor,
#                            corrector, window sum)
#   phase wrap / 4 steps:    floor, sub, convert, add
# ---------------------------------------------------------------------------
PEAK_SLOTS = 256 * 4 * 16 * 2.4e9
W_MUL64 = 4.0   # v_mad_u64_u32 issue cost in full-rate slots
W_TRANS = 4.0   # v_sin/v_cos/v_log/v_sqrt issue cost in full-rate slots


def jj_slots_per_path_step(w_mul=W_MUL64, w_trans=W_TRANS):
    philox = (20 * w_mul + 40) / 4
    box_muller = (2 + 1 + 2 + 2 + 1 + 2 + 3 * w_trans + w_trans) / 2
    heun = 13 + 2 * w_trans
    wrap = 4 / 4
    return philox + box_muller + heun + wrap


def jj_flops_per_path_step():
    """FP32 floating-point operations (transcendentals count 1)."""
    return (2 + 1 + 2 + 4 + 2) / 2 + 13 + 2 + 1


def cpu_baseline(seed, target_s):
    """FP64 oracle on 16 scan points (4 x 4 sub-grid) x 256 paths x the full
    2*10^5 steps, all host threads."""
    import oracle
    qs = [128 * i + j for i in (0, 42, 85, 127) for j in (0, 42, 85, 127)]
    n_paths = 256
    pts = sde_inputs.jj_scan(n_paths=n_paths, indices=qs)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    # scale the sample down if this host is slow (about target_s seconds)
    probe = [dict(pts[0], n_paths=64, n_steps=20000, n_transient=10000)]
    t0 = time.perf_counter()
    oracle.jj_integrate(probe, seed, point_ids=[qs[0]], n_threads=threads)
    rate_est = 64 * 20000 / (time.perf_counter() - t0)
    full = len(qs) * n_paths * 200000
    if full / rate_est > target_s:
        n_paths = max(16, int(n_paths * target_s * rate_est / full) // 16 * 16)
        pts = sde_inputs.jj_scan(n_paths=n_paths, indices=qs)
    t0 = time.perf_counter()
    oracle.jj_integrate(pts, seed, point_ids=qs, n_threads=threads)
    dt = time.perf_counter() - t0
    work = len(qs) * n_paths * 200000
    return {"value": work / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(qs)} scan points (4x4 sub-grid) x {n_paths} paths x 2e5 Heun steps, "
                      f"FP64, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--model-steps", type=int, default=200000,
                    help="Heun steps per path (the workload uses 2e5; smaller only for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the JJ scan would shard "
              "by points across GPUs with no exchange but a final gather, which this build does not "
              "launch.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0903_3852_amd as sde

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    seed = sde_inputs.seed_of(2)
    n_steps = args.model_steps
    pts = sde.make_points(sde_inputs.jj_scan(n_steps=n_steps, n_transient=n_steps // 2))
    path_steps = 16384 * 1024 * n_steps
    ps = torch.empty((16384, 2), dtype=torch.float64, device=dev)
    ctx = sde.sde_create(0)
    run = sde.make_run(seed)
    stream = torch.cuda.current_stream()

    for w in range(args.warmup):
        sde.sde_jj_integrate(ctx, pts, run, point_sums=ps)
        torch.cuda.synchronize()
        print(f"warmup {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        sde.sde_jj_integrate(ctx, pts, run, point_sums=ps)
        ends[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sde.sde_check(ctx)
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kernel_s = float(np.mean(ms)) / 1e3
    sums = ps.cpu().numpy()
    assert np.all(np.isfinite(sums))
    print(f"timed {args.steps} steps: {ms} ms per step, wall {wall:.2f} s", file=sys.stderr, flush=True)

    value = path_steps * args.steps / wall
    slots = jj_slots_per_path_step()
    achieved = slots * path_steps / kernel_s / 1e12
    out = {
        "metric": "path-steps/s (Josephson-junction scan, stochastic Heun)",
        "value": value, "unit": "path-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "jj_scan", "points": 16384, "paths_per_point": 1024,
                   "heun_steps": n_steps, "transient": n_steps // 2, "dt": "2pi/omega/200",
                   "path_steps_per_step": path_steps},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_SLOTS / 1e12,
                     "unit": "T VALU-slots/s", "frac": achieved * 1e12 / PEAK_SLOTS,
                     "traffic": None},
        "fp32_tflops": jj_flops_per_path_step() * path_steps / kernel_s / 1e12,
        "kernel_ms": float(np.mean(ms)),
        "mean_v_range": [float(sums[:, 0].min() / 1024), float(sums[:, 0].max() / 1024)],
    }
    sde.sde_destroy(ctx)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(seed, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = value / cb["value"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
