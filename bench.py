"""Benchmark of the SDE-ensemble hot path on one MI355X.

Default workload (--workload jj_scan): the Josephson-junction (f, D) scan --
128 x 128 points (f = 0.5 i/127, D = 10^(-4 + 3 j/127)), 1024 paths per
point, 2*10^5 stochastic-Heun steps of dt = 2 pi/omega/200 (10^5
transient), FP32 state with FP64 <v> accumulation, all 16384 points in one
persistent launch.  A benchmark "step" is one such full integration
(3.36e12 path-steps) with the parameters resident before timing starts.

The other workloads (--workload kuramoto_*) time the Kuramoto kernels on
their own configurations; the default run also reports short measurements
of them under "kuramoto".

Prints one JSON line: throughput, the roofline fraction of the dominant
kernel (timed with HIP events on the stream it runs on) and the FP64 CPU
oracle timed on a bounded sample of the same workload; each Kuramoto leg
carries the oracle timed on a sample of its own configuration.
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import sde_inputs  # noqa: E402

_T0 = time.time()


def progress(msg):
    """A progress line on stderr (long legs print one at least every minute)."""
    print(f"[{time.time() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)

# ---------------------------------------------------------------------------
# ALU roofline.  Peak: the FP32 vector rate, 256 CUs x 4 SIMDs x 32 FP32 lanes
# x 2.4 GHz = 7.86e13 lane-operations per second (157.3 TFLOP/s as FMAs), one
# wave64 FP32 add / mul / fma or 32-bit integer operation per 2 SIMD cycles
# without packed instructions.  The forms with an SGPR operand,
# v_mad_u64_u32, v_mul_hi_u32, conversions, floor and FP64 add/fma run at half
# that rate, the transcendentals (v_sin, v_cos, v_log, v_sqrt) at a quarter.
# Algorithmic work is counted in units of the peak's lane-operation: W_FULL =
# 1, W_HALF = 2, W_TRANS = 4, each operation the method needs counted once in
# its cheapest form.  (--workload valu_costs times each form alone: streams of
# one full-rate form take 2.9-3.8 cycles per instruction, the half-rate forms
# 4.4-5.1, the transcendentals 8.3-8.4; a mixed stream issues faster, the
# transcendentals overlapping other work, so the fractions are against the
# published peak and do not flatter the kernels.)
# ---------------------------------------------------------------------------
PEAK_FMA_LANES = 256 * 4 * 32 * 2.4e9
PEAK_MFMA_16BIT = 2.5e15           # dense bf16 / fp16 MFMA FLOP/s
PEAK_MFMA_FP32 = 157.3e12          # FP32 MFMA FLOP/s
W_FULL = 1.0
W_HALF = 2.0
W_TRANS = 4.0
# Philox4x32-10 per block of four steps: 10 rounds x (2 wide products, each a
# half-rate v_mad_u64_u32, and 2 three-way xors, each one v_bitop3_b32).
PHILOX_BLOCK = 10 * (2 * W_HALF + 2 * W_FULL)
# Box-Muller per pair of Gaussians: u1 = shift, add, convert, scale; u2 =
# shift, convert, scale; log2, times c2, sqrt; cos, sin and two products.
BOX_MULLER_PAIR = (3 * W_FULL + W_HALF) + (2 * W_FULL + W_HALF) + (2 * W_TRANS + W_FULL) + (2 * W_TRANS + 2 * W_FULL)
# Noise per path (or oscillator) and step: a quarter of a Philox block, half a pair.
NOISE_OPS = PHILOX_BLOCK / 4 + BOX_MULLER_PAIR / 2


def jj_ops_per_path_step():
    """One stochastic-Heun path-step of Eq. 1: noise, 2 sin + 13 FP32 (two
    drift evaluations, predictor, corrector, window sum), phase wrap per four
    steps (floor, subtract, convert, add)."""
    return NOISE_OPS + 13 * W_FULL + 2 * W_TRANS + (2 * W_HALF + 2 * W_FULL) / 4


def jj_valu_instr_per_path_step():
    """VALU instructions per path-step the method needs (a transcendental
    counts 1): Philox 10, Box-Muller 7, Heun 15, wrap 1."""
    return 40 / 4 + 14 / 2 + 15 + 4 / 4


def jj_flops_per_path_step():
    """FP32 floating-point operations (a transcendental counts 1)."""
    return (5 + 4) / 2 + 13 + 2 + 2 / 4


def mf_ops_per_osc_step(heun):
    """Mean-field Kuramoto per oscillator-step: noise; per stage sin + cos
    and one add into each of the two sums; drift (3) and update (2 + 3 in
    the corrector); wrap (floor, subtract)."""
    stage = 2 * W_TRANS + 2 * W_FULL
    if heun:
        return NOISE_OPS + 2 * stage + 3 + 2 + 3 + 3 + W_HALF + W_FULL
    return NOISE_OPS + stage + 3 + 2 + W_HALF + W_FULL


def mfs_ops_per_osc_step(heun):
    """Streamed mean field per oscillator-step: Philox every step and one
    Gaussian; sin + cos evaluated 4 times (Heun: theta, tt twice, theta') or
    twice (Euler), two adds into the sums per stage; drift, update and wrap."""
    noise = PHILOX_BLOCK + (3 * W_FULL + W_HALF) + (2 * W_FULL + W_HALF) + (2 * W_TRANS + W_FULL) + W_TRANS + W_FULL
    trans = (8 if heun else 4) * W_TRANS
    sums = (2 if heun else 1) * 2 * W_FULL
    return noise + trans + sums + (12 if heun else 7)


def mfs_bytes_per_osc_step(heun):
    """HBM bytes per oscillator-step of the streamed mean field: Heun reads
    theta, omega and writes tt, carry; then reads tt, carry and writes theta
    (7 words); Euler-Maruyama reads theta, omega and writes theta (3)."""
    return 4 * (7 if heun else 3)


PEAK_HBM = 8.0e12
# Measured HBM bytes per oscillator-step of the streamed mean field (Fig. 4),
# from profiles/kuramoto_fig4_hbm_counters.md; valid for that kernel source.
FIG4_TRAFFIC_PER_OSC_STEP = 28.05
FIG4_TRAFFIC_SOURCE_SHA1 = "82fa5aac87989d0a864b0ddad5c1b282e932dd53"


def _source_sha1(*files):
    h = hashlib.sha1()
    for f in files:
        with open(os.path.join(ROOT, "paper_0903_3852_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# HBM traffic of the JJ kernel per launch, from profiles/jj_scan_hbm_counters.md
# (FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00, copy-calibrated), and its VALU
# counters per path-step, from profiles/jj_scan_valu_counters.md.  Only valid
# for the kernel source they were measured on.
JJ_TRAFFIC_BYTES = (2 * 3547.2 + 6612.1) * 1024
JJ_TRAFFIC_SOURCE_SHA1 = "ca5065025955cec058718be06875fb2e71ce5666"
JJ_VALU_COUNTERS = {"valu_instructions_per_path_step": 34.28, "transcendental_per_path_step": 4.00,
                    "salu_instructions_per_path_step": 8.08, "valu_instructions_per_simd_cycle": 0.262,
                    "source": "profiles/jj_scan_valu_counters.md"}


# VALU counters of the Kuramoto kernels, valid while the kernel's section of
# kuramoto.hip and device_common.h are the ones they were taken on.
KURA_VALU_COUNTERS = {
    "kuramoto_tiled": ({"valu_instructions_per_pair_term": 3.08, "transcendental_per_pair_term": 1.00,
                        "valu_instructions_per_simd_cycle": 0.187,
                        "source": "profiles/kuramoto_tiled_valu_counters.md"},
                       ("-- TILED ------", "-- host --"), "99154c35b9150737c63b10052e2fb4d746117639"),
    "kuramoto_mf": ({"valu_instructions_per_oscillator_stage": 29.1, "transcendental_per_oscillator_stage": 3.07,
                     "valu_instructions_per_simd_cycle": 0.108, "source": "profiles/kuramoto_meanfield_counters.md"},
                    ("-- MF ------", "-- MF, two realizations per workgroup --"), "fddd8c97c34c8a31a73975c59e0ff3a61eb17c25"),
}


def _section_sha1(path, first, last):
    """SHA-1 of the lines of `path` from the one containing `first` to the
    next one containing `last`, followed by device_common.h."""
    out, on = [], False
    with open(path) as fh:
        for line in fh.read().split("\n"):
            if first in line:
                on = True
            if on:
                out.append(line)
            if on and last in line and first not in line:
                break
    h = hashlib.sha1(("\n".join(out) + "\n").encode())
    with open(os.path.join(ROOT, "paper_0903_3852_amd", "csrc", "device_common.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def kura_counters(name):
    """The VALU counters of workload `name`'s kernel if its source is the one they were taken on."""
    if name not in KURA_VALU_COUNTERS:
        return None
    rec, (first, last), sha = KURA_VALU_COUNTERS[name]
    return rec if _section_sha1(os.path.join(ROOT, "paper_0903_3852_amd", "csrc", "kuramoto.hip"), first,
                                last) == sha else None


def _jj_source_sha1():
    h = hashlib.sha1()
    for f in ("jj.hip", "device_common.h"):
        with open(os.path.join(ROOT, "paper_0903_3852_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_one_core(seed):
    """The paper's CPU methodology (one core of its host): the FP64 oracle on
    one thread, one point (the single-point parameters) x 1024 paths x 10^4
    Heun steps."""
    import oracle
    pts = sde_inputs.jj_single(n_paths=1024, n_steps=10000)
    t0 = time.perf_counter()
    oracle.jj_integrate(pts, seed, n_threads=1)
    dt = time.perf_counter() - t0
    return {"value": 1024 * 10000 / dt, "unit": "path-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"1 point x 1024 paths x 1e4 Heun steps, FP64, one thread, {dt:.2f} s"}


def cpu_baseline_jj(seed, target_s):
    """FP64 oracle on 64 scan points (f and D indices multiples of 16, an
    8 x 8 sub-grid) x 1024 paths x the full 2*10^5 steps (fewer paths if
    this host would take longer than target_s), all host threads.  Returns
    (baseline record, oracle result, qs, paths)."""
    import oracle
    qs = [128 * i + j for i in range(0, 128, 16) for j in range(0, 128, 16)]
    n_paths = 1024
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    probe = [sde_inputs.jj_scan(n_paths=64, n_steps=20000, n_transient=10000, indices=[qs[0]])[0]]
    t0 = time.perf_counter()
    oracle.jj_integrate(probe, seed, point_ids=[qs[0]], n_threads=threads)
    rate_est = 64 * 20000 / (time.perf_counter() - t0)
    if len(qs) * n_paths * 200000 / rate_est > target_s:
        n_paths = max(16, int(target_s * rate_est / (len(qs) * 200000)) // 16 * 16)
    pts = sde_inputs.jj_scan(n_paths=n_paths, indices=qs)
    t0 = time.perf_counter()
    ref = oracle.jj_integrate(pts, seed, point_ids=qs, n_threads=threads)
    dt = time.perf_counter() - t0
    work = len(qs) * n_paths * 200000
    rec = {"value": work / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(qs)} scan points (8x8 sub-grid, indices multiples of 16) x {n_paths} paths x 2e5 "
                     f"Heun steps, FP64, {dt:.1f} s",
           "host": {"nproc": os.cpu_count(), "cpu_model": _cpu_model()},
           "one_core": cpu_baseline_one_core(seed)}
    return rec, ref, qs, n_paths


def bench_jj(args, sde, torch, dev):
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
    stats = sde.sde_get_stats(ctx)
    sde.sde_destroy(ctx)
    ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    kernel_s = float(np.mean(ms)) / 1e3
    sums = ps.cpu().numpy()
    assert np.all(np.isfinite(sums))
    print(f"timed {args.steps} steps: {ms} ms per step, wall {wall:.2f} s", file=sys.stderr, flush=True)
    ops = jj_ops_per_path_step()
    achieved = ops * path_steps / kernel_s
    same_source = _jj_source_sha1() == JJ_TRAFFIC_SOURCE_SHA1
    traffic = JJ_TRAFFIC_BYTES if (same_source and n_steps == 200000) else None
    out = {
        "metric": "path-steps/s (Josephson-junction scan, stochastic Heun)",
        "value": path_steps * args.steps / wall, "unit": "path-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "jj_scan", "points": 16384, "paths_per_point": 1024,
                   "heun_steps": n_steps, "transient": n_steps // 2, "dt": "2pi/omega/200",
                   "path_steps_per_step": path_steps},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FMA_LANES / 1e12,
                     "unit": "T lane-op units/s", "frac": achieved / PEAK_FMA_LANES,
                     "traffic": traffic, "ops_per_path_step": ops,
                     "valu_instructions_per_path_step_method": jj_valu_instr_per_path_step(),
                     "counters": JJ_VALU_COUNTERS if same_source else None,
                     "kernel": f"jj_persistent_kernel<float, {stats['jj_paths_per_lane']}, HEUN, inertial, sin>"},
        "launch": {"paths_per_lane": stats["jj_paths_per_lane"], "graph_replayed": stats["graph_replayed"],
                   "work_items": stats["work_items"]},
        "fp32_tflops": jj_flops_per_path_step() * path_steps / kernel_s / 1e12,
        "kernel_ms": float(np.mean(ms)),
    }
    if not args.no_cpu_baseline:
        cb, ref, qs, n_paths = cpu_baseline_jj(seed, args.cpu_seconds)
        out["cpu_baseline"] = cb
        out["gpu_over_cpu"] = out["value"] / cb["value"]
        if n_steps == 200000:
            # parity of the timed run at the sample points: the GPU mean over
            # 1024 paths against the oracle's mean over the first n_paths of
            # the same paths (same Philox streams)
            g = sums[qs, 0] / 1024
            o = ref["point_sums"][:, 0] / n_paths
            var_o = np.maximum(ref["point_sums"][:, 1] / n_paths - o * o, 0.0)
            se = np.sqrt(var_o / n_paths + var_o / 1024)
            ratio = np.abs(g - o) / (3 * se + 1e-4)
            out["parity"] = {"points": len(qs), "max_abs_diff_vmean": float(np.abs(g - o).max()),
                             "max_diff_over_3se_plus_1e-4": float(ratio.max()), "ok": bool(ratio.max() <= 1.0)}
    return out


def bench_jj_batch(args, sde, torch, dev):
    """The uneven batch: 2048 random points (a ~ U[2,6], omega ~ U[3,7],
    f ~ U[0,0.5], log10 D ~ U[-4,-1], gamma ~ U[0.5,1.5]) with paths in
    {256..8192} and steps in {5e4..4e5} (half transient), one persistent
    launch.  Tail efficiency = the time the same path-steps would take at
    the rate of the uniform scan kernel / the measured time."""
    pts_l = sde_inputs.jj_batch()
    pts = sde.make_points(pts_l)
    work = sum(p["n_paths"] * p["n_steps"] for p in pts_l)
    ps = torch.empty((len(pts_l), 2), dtype=torch.float64, device=dev)
    acc = torch.empty(sum(p["n_paths"] for p in pts_l), dtype=torch.float64, device=dev)
    ctx = sde.sde_create(0)
    run = sde.make_run(sde_inputs.seed_of(5))
    stream = torch.cuda.current_stream()
    sde.sde_jj_integrate(ctx, pts, run, acc=acc, point_sums=ps)  # warm-up (tunes, records the graph)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    sde.sde_jj_integrate(ctx, pts, run, acc=acc, point_sums=ps)
    e.record(stream)
    torch.cuda.synchronize()
    st = sde.sde_get_stats(ctx)
    sde.sde_check(ctx)
    sde.sde_destroy(ctx)
    t = s.elapsed_time(e) / 1e3
    ops = jj_ops_per_path_step()
    rec = {"workload": "jj_batch", "points": len(pts_l), "path_steps": work, "seconds": t,
           "path_steps_per_s": work / t, "paths_per_lane": st["jj_paths_per_lane"],
           "work_items": st["work_items"], "graph_replayed": st["graph_replayed"],
           "roofline": {"bound": "alu", "achieved": ops * work / t / 1e12, "peak": PEAK_FMA_LANES / 1e12,
                        "unit": "T lane-op units/s", "frac": ops * work / t / PEAK_FMA_LANES,
                        "traffic": None}}
    if not getattr(args, "no_cpu_baseline", True):
        # the FP64 oracle beside it: the first 8 points, 128 paths each, all their steps, under their
        # batch indices (the same noise streams as the GPU's paths 0..127 of those points)
        import oracle
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        sample = [dict(p, n_paths=128) for p in pts_l[:8]]
        t0 = time.perf_counter()
        ref = oracle.jj_integrate(sample, sde_inputs.seed_of(5), point_ids=list(range(8)), n_threads=threads)
        dt = time.perf_counter() - t0
        w = sum(p["n_paths"] * p["n_steps"] for p in sample)
        rec["cpu_baseline"] = {"value": w / dt, "unit": "path-steps/s", "cores": threads, "kind": "oracle",
                             "sample": f"8 batch points x 128 paths x their 5e4-4e5 steps, FP64, {dt:.1f} s",
                             "gpu_over_cpu": work / t / (w / dt)}
        # the timed launch against the oracle on those paths: paired
        # time-averaged velocities, |mean difference| <= 3 SE + 1e-4 per point
        a = acc.cpu().numpy()
        first = np.concatenate([[0], np.cumsum([p["n_paths"] for p in pts_l])[:-1]])
        worst, dmax = 0.0, 0.0
        for q, p in enumerate(sample):
            W = p["n_steps"] - p["n_transient"]
            d = a[first[q]:first[q] + 128] / W - ref["acc"][128 * q:128 * (q + 1)] / W
            se = d.std(ddof=1) / np.sqrt(d.size)
            worst = max(worst, abs(d.mean()) / (3 * se + 1e-4))
            dmax = max(dmax, abs(d.mean()))
        rec["parity"] = {"against": "FP64 oracle", "points": 8, "paths_per_point": 128,
                         "max_abs_diff_vmean": dmax, "max_diff_over_3se_plus_1e-4": worst, "ok": bool(worst <= 1.0)}
    return rec


SPREAD_MAX = 0.02                          # fall back to simulation above this ensemble spread
SURR_CENTER = [4.0, 5.0, 0.25, -2.5, 1.0]   # features (a, omega, f, log10 D, gamma) -> [-1, 1]
SURR_SCALE = [2.0, 2.0, 0.25, 1.5, 0.5]


# the second surrogate distribution: the paper's potential around Fig. 2
ANM_CENTER = [4.25, 5.0, 0.0, -3.0, 0.95]
ANM_SCALE = [0.75, 1.0, 0.3, 1.0, 0.25]
SURR_VARIANTS = {
    # params generator, feature centre/scale, potential, steps per drive period, queries in the timed
    # scan, training points, training schedule (epochs, learning rate) in order, Adam's state carried
    # from one stage to the next
    "batch": (sde_inputs.jj_random_params, SURR_CENTER, SURR_SCALE, 0, 200, 1000000, 100000, ((30, 1e-3),)),
    "anm": (sde_inputs.jj_anm_params, ANM_CENTER, ANM_SCALE, 1, 100, 100000, 1000000,
            ((150, 1e-3), (50, 3e-4), (50, 1e-4), (50, 3e-5))),
}


def _surr_points(sde, P, paths, steps, potential=0, spp=200):
    return sde.make_points_np(m=1.0, gamma=P[:, 4], a=P[:, 0], omega=P[:, 1], f=P[:, 2], D=P[:, 3],
                              n_paths=paths, steps_per_period=spp, n_steps=steps, n_transient=steps // 2,
                              potential=potential)


def bench_surrogate(args, sde, torch, dev, variant="batch"):
    """The learned <v> surrogate: labels simulated by the integrator (512
    paths x 1e5 steps, half transient), 5 members of 5-256-256-256-1 trained
    on the GPU (1e5 points x 30 epochs at lr 1e-3; for "anm" 1e6 points x 300
    epochs, the learning rate stepped 1e-3, 3e-4, 1e-4, 3e-5), and a scan
    that falls back to simulation where the members' spread exceeds 0.02.
    Reported: error against 4096 held-out points simulated at 4096 paths at
    that threshold (and at every candidate of 0.005 ... 0.1, and without
    fallback), and the timed scan; beside them the largest candidate whose
    error on 2048 validation points is within 1e-2, and its timed scan.  The
    plain method simulates every query with the same 512 x 1e5 budget; its
    time is measured on 1e4 queries and scaled linearly (the queries are
    independent).  variant
    "batch": the batch parameter distribution with the -sin(phi) drift
    (dt = 2pi/omega/200), 1e6 queries; "anm": the paper's potential around
    its Fig. 2 point (dt = 0.01 drive period), where <v> varies in sign and
    size, 1e5 queries."""
    gen, center, scale, potential, spp, n_query, n_train, schedule = SURR_VARIANTS[variant]
    ctx = sde.sde_create(0)
    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def simulate(P, paths, steps, seed):
        pts = _surr_points(sde, P, paths, steps, potential, spp)
        ps = torch.empty((len(P), 2), dtype=torch.float64, device=dev)
        s, e = ev(), ev()
        s.record(stream)
        sde.sde_jj_integrate(ctx, pts, sde.make_run(seed), point_sums=ps)
        e.record(stream)
        torch.cuda.synchronize()
        return ps.cpu().numpy()[:, 0] / paths, s.elapsed_time(e) / 1e3

    seed = sde_inputs.seed_of(5) + (0 if variant == "batch" else 1000)
    Ptr = gen(n_train, seed + 50)
    ytr, t_labels = simulate(Ptr, 512, 100000, seed + 51)
    progress(f"surrogate {variant}: {n_train} training labels in {t_labels:.1f} s")
    Pho = gen(4096, seed + 60)
    yho, _ = simulate(Pho, 4096, 100000, seed + 61)
    Pva = gen(2048, seed + 65)  # validation set: picks the spread threshold
    yva, _ = simulate(Pva, 4096, 100000, seed + 66)
    progress(f"surrogate {variant}: held-out and validation labels done")

    def feats(P):
        X = P.astype(np.float64).copy()
        X[:, 3] = np.log10(X[:, 3])
        return torch.from_numpy(X.astype(np.float32)).to(dev)

    sur = sde.sde_surrogate_create(ctx, [5, 256, 256, 256, 1], 5, seed + 70)
    sde.sde_surrogate_set_scaling(sur, sde.make_scaling(center, scale, float(ytr.mean()), float(ytr.std()), 0))
    Xtr, Ytr = feats(Ptr), torch.from_numpy(ytr.astype(np.float32)).to(dev)
    t0 = time.perf_counter()
    curve = []
    for k, (epochs_k, lr_k) in enumerate(schedule):
        curve += list(sde.sde_surrogate_train(sur, Xtr, Ytr, sde.make_train_opts(epochs_k, 1024, lr=lr_k,
                                                                                 shuffle_seed=seed + 71 + k)))
        progress(f"surrogate {variant}: training stage {k + 1}/{len(schedule)} ({epochs_k} epochs at lr {lr_k:g})")
    t_train = time.perf_counter() - t0
    # the spread threshold: the largest candidate whose validation error (scan
    # with fallback against 4096-path labels) is within 1e-2
    cands = (0.005, 0.01, 0.02, 0.05, 0.1)

    def scan_err(P, y, smax, seed_):
        q = _surr_points(sde, P, 512, 100000, potential, spp)
        vv = torch.empty(len(P), dtype=torch.float64, device=dev)
        uu = torch.empty(len(P), dtype=torch.uint8, device=dev)
        sde.sde_surrogate_scan(sur, q, smax, sde.make_run(seed_), vv, uu)
        return np.abs(vv.cpu().numpy() - y), uu.cpu().numpy(), vv.cpu().numpy()

    val = [(c, float(scan_err(Pva, yva, c, seed + 75)[0].mean())) for c in cands]
    chosen = max([c for c, m in val if m <= 1e-2], default=cands[0])
    # held-out error of the scan (prediction or fallback simulation) at every
    # candidate, and without fallback
    tradeoff = []
    for smax in cands + (1e9,):
        e_s, u_s, _ = scan_err(Pho, yho, smax, seed + 80)
        tradeoff.append({"spread_max": smax if smax < 1e8 else None, "mae": float(e_s.mean()),
                         "p95": float(np.quantile(e_s, 0.95)), "fallback_share": float(u_s.mean())})
    # the headline threshold is the configured spread_max = 0.02
    err, uho, vho = scan_err(Pho, yho, SPREAD_MAX, seed + 80)
    r2 = 1.0 - np.mean((vho - yho) ** 2) / np.var(yho)
    # the timed scan at 0.02, and at the validated threshold
    Pq = gen(n_query, seed + 90)
    queries = _surr_points(sde, Pq, 512, 100000, potential, spp)
    vq = torch.empty(n_query, dtype=torch.float64, device=dev)
    uq = torch.empty(n_query, dtype=torch.uint8, device=dev)
    sde.sde_surrogate_scan(sur, _surr_points(sde, Pq[:1000], 512, 100000, potential, spp), SPREAD_MAX,
                           sde.make_run(seed + 91), vq, uq)  # warm-up

    def timed_scan(smax):
        t0 = time.perf_counter()
        st_ = sde.sde_surrogate_scan(sur, queries, smax, sde.make_run(seed + 91), vq, uq)
        return st_, time.perf_counter() - t0

    st, t_scan = timed_scan(SPREAD_MAX)
    st_v, t_scan_v = timed_scan(chosen)
    # the plain method on a 1e4-query subset, scaled to 1e6
    _, t_plain_sub = simulate(Pq[:10000], 512, 100000, seed + 91)
    t_plain = t_plain_sub * n_query / 10000
    sde.sde_surrogate_destroy(sur)
    sde.sde_destroy(ctx)
    progress(f"surrogate {variant}: scans done")
    return {"workload": "jj_surrogate" if variant == "batch" else "jj_surrogate_anm",
            "potential": "-sin(phi)" if potential == 0 else "sin(2 pi x)",
            "train_points": n_train, "label_budget": "512 paths x 1e5 steps",
            "label_seconds": t_labels, "train_seconds": t_train,
            "schedule": [{"epochs": e_, "lr": l_} for e_, l_ in schedule],
            "loss_first_last": [float(curve[0]), float(curve[-1])],
            "holdout": {"points": 4096, "paths": 4096, "mae": float(err.mean()),
                        "p95": float(np.quantile(err, 0.95)), "max": float(err.max()), "r2": r2,
                        "label_std": float(yho.std()), "mae_of_zero": float(np.abs(yho).mean()),
                        "fallback": int(uho.sum()), "spread_tradeoff": tradeoff},
            "validation": {"points": 2048, "paths": 4096, "mae_by_spread_max": val, "chosen_spread_max": chosen},
            "scan": {"queries": n_query, "spread_max": SPREAD_MAX, "fallback": int(st["n_fallback"]),
                     "fallback_share": int(st["n_fallback"]) / n_query,
                     "predict_ms": st["predict_ms"], "fallback_ms": st["fallback_ms"],
                     "total_s": t_scan, "queries_per_s": n_query / t_scan},
            "plain_simulation_s": t_plain, "speedup": t_plain / t_scan,
            "scan_validated_threshold": {"spread_max": chosen, "fallback": int(st_v["n_fallback"]),
                                         "total_s": t_scan_v, "speedup": t_plain / t_scan_v}}


def bench_fig2(args, sde, torch, dev):
    """The paper's Fig. 2 ensemble: 2^19 paths of Eq. 1 with V(x) = sin(2 pi x)
    at a = 4.2, gamma = 0.9, omega = 4.9, D = 0.001, f = 0.1, dt = 0.01 of the
    drive period, 2000 periods (2*10^5 Heun steps), then the coarse-grained
    position histogram (200 bins of one period, centred on the ensemble), and
    the density over time from every path's period streamed once per drive
    period.  The paper's single-precision run took 20 s on its GPU, including
    writing every particle position to disk: context, not a target."""
    pts = sde_inputs.jj_fig2()
    P, n = pts[0]["n_paths"], pts[0]["n_steps"]
    th = torch.empty(P, dtype=torch.float32, device=dev)
    wd = torch.empty(P, dtype=torch.int32, device=dev)
    v = torch.empty(P, dtype=torch.float32, device=dev)
    acc = torch.empty(P, dtype=torch.float64, device=dev)
    counts = torch.zeros(202, dtype=torch.int64, device=dev)
    ctx = sde.sde_create(0)
    run = sde.make_run(sde_inputs.seed_of(20))
    stream = torch.cuda.current_stream()
    sde.sde_jj_integrate(ctx, [dict(pts[0], n_steps=100)], run, th, wd, v, acc)  # warm-up
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    sde.sde_jj_integrate(ctx, pts, run, th, wd, v, acc)
    e.record(stream)
    torch.cuda.synchronize()
    t = s.elapsed_time(e) / 1e3
    parity = None
    if not getattr(args, "no_cpu_baseline", True):
        # error against the FP64 oracle: one step from the run's final state,
        # the first 8192 paths (x = theta + winding periods, v)
        import oracle
        st1 = tuple(x.clone() for x in (th, wd, v, acc))
        sde.sde_jj_integrate(ctx, [dict(pts[0], n_steps=1)],
                             sde.make_run(sde_inputs.seed_of(20), step0=n, init=sde.SDE_INIT_FROM_STATE, sync=1), *st1)
        k = 8192
        x0 = th[:k].cpu().double().numpy() + wd[:k].cpu().double().numpy()
        ref = oracle.jj_integrate([dict(pts[0], n_paths=k, n_steps=1)], sde_inputs.seed_of(20), step0=n,
                                  state=(x0, v[:k].cpu().double().numpy(), np.zeros(k)))
        x1 = st1[0][:k].cpu().double().numpy() + st1[1][:k].cpu().double().numpy()
        e_x = np.abs(x1 - ref["phi"]) / np.maximum(np.abs(ref["phi"]), 1.0)
        e_v = np.abs(st1[2][:k].cpu().double().numpy() - ref["v"]) / np.maximum(np.abs(ref["v"]), 1.0)
        worst = float(max(e_x.max(), e_v.max()))
        parity = {"against": "FP64 oracle", "what": f"one Heun step from the state at step {n}, paths 0..{k - 1}",
                  "max_rel_err": worst, "bound": 1e-5, "ok": bool(worst <= 1e-5)}
        del st1
    # the density over time (Fig. 2, left panel): every path's winding after
    # every drive period (100 steps), 2000 rows streamed into HBM during the
    # run, then the histograms of all rows in one call (fixed window of 600
    # periods around the start)
    every = 100
    rows = n // every
    rec = torch.empty((rows, P), dtype=torch.int32, device=dev)
    st2 = tuple(torch.empty_like(x) for x in (th, wd, v, acc))
    sde.sde_jj_integrate_recorded(ctx, [dict(pts[0], n_steps=100)], run, every, rec[:1], *st2)  # warm-up
    torch.cuda.synchronize()
    s.record(stream)
    sde.sde_jj_integrate_recorded(ctx, pts, run, every, rec, *st2)
    e.record(stream)
    torch.cuda.synchronize()
    t_rec = s.elapsed_time(e) / 1e3
    xlo, nbw = -400, 600
    dens = torch.empty((rows, nbw + 2), dtype=torch.int64, device=dev)
    sde.sde_position_histograms(ctx, rec[:2], xlo, nbw, dens[:2])  # warm-up
    torch.cuda.synchronize()
    s.record(stream)
    sde.sde_position_histograms(ctx, rec, xlo, nbw, dens)
    e.record(stream)
    torch.cuda.synchronize()
    t_hist = s.elapsed_time(e) / 1e3
    same = bool(torch.equal(st2[1], wd) and torch.equal(st2[0], th) and torch.equal(rec[-1], wd))
    dn = dens.cpu().numpy()
    del rec, dens
    centre = xlo + np.arange(nbw) + 0.5
    inner = dn[:, 1:nbw + 1].astype(np.float64)
    mean_t = (inner * centre).sum(axis=1) / inner.sum(axis=1)
    sd_t = np.sqrt((inner * centre ** 2).sum(axis=1) / inner.sum(axis=1) - mean_t ** 2)
    density = {"record_every_steps": every, "rows": rows, "bytes_streamed": rows * P * 4,
               "seconds_recorded_run": t_rec, "recording_overhead": t_rec / t - 1.0,
               "histogram_seconds_all_rows": t_hist, "window": [xlo, xlo + nbw],
               "outside_window_max": int((dn[:, 0] + dn[:, nbw + 1]).max()),
               "same_trajectory_as_plain_run": same,
               "mean_sd_at_periods": {str(k): [round(float(mean_t[k - 1]), 3), round(float(sd_t[k - 1]), 3)]
                                      for k in (10, 100, 500, 1000, 2000)}}
    # the same ensemble in double precision (the paper's precision study)
    th64 = torch.empty(P, dtype=torch.float64, device=dev)
    wd64 = torch.empty(P, dtype=torch.int32, device=dev)
    v64 = torch.empty(P, dtype=torch.float64, device=dev)
    acc64 = torch.empty(P, dtype=torch.float64, device=dev)
    sde.sde_jj_integrate_f64(ctx, [dict(pts[0], n_steps=100)], run, th64, wd64, v64, acc64)  # warm-up
    torch.cuda.synchronize()
    s.record(stream)
    sde.sde_jj_integrate_f64(ctx, pts, run, th64, wd64, v64, acc64)
    e.record(stream)
    torch.cuda.synchronize()
    t64 = s.elapsed_time(e) / 1e3
    x0 = int(wd64.median().item()) - 100
    counts64 = torch.zeros(202, dtype=torch.int64, device=dev)
    sde.sde_position_histogram(ctx, wd, x0, 200, counts)
    sde.sde_position_histogram(ctx, wd64, x0, 200, counts64)
    torch.cuda.synchronize()
    sde.sde_check(ctx)
    sde.sde_destroy(ctx)
    h, h64 = counts.cpu().numpy(), counts64.cpu().numpy()
    keep = (h + h64) >= 10
    chi2 = float((((h[keep] - h64[keep]) ** 2) / (h[keep] + h64[keep])).sum())
    from scipy import stats
    vb, vb64 = acc.cpu().numpy() / n, acc64.cpu().numpy() / n
    x = th.cpu().double().numpy() + wd.cpu().double().numpy()
    return {"workload": "jj_fig2", "potential": "sin(2 pi x)", "paths": P, "heun_steps": n,
            "seconds": t, "path_steps_per_s": P * n / t,
            "mean_velocity": float(vb.mean()), "mean_velocity_se": float(vb.std(ddof=1) / np.sqrt(P)),
            "position_mean": float(x.mean()), "position_sd": float(x.std()),
            "histogram": {"x0": x0, "bins": 200, "underflow": int(h[0]), "overflow": int(h[201]),
                          "occupied_bins": int(np.count_nonzero(h[1:201])), "max_bin": int(h[1:201].max())},
            "density_over_time": density,
            "parity": parity,
            "fp64": {"seconds": t64, "path_steps_per_s": P * n / t64, "fp64_over_fp32_time": t64 / t,
                     "mean_velocity": float(vb64.mean()), "mean_velocity_se": float(vb64.std(ddof=1) / np.sqrt(P)),
                     "histogram_chi2": chi2, "histogram_dof": int(keep.sum() - 1),
                     "histogram_p": float(stats.chi2.sf(chi2, keep.sum() - 1)),
                     "same_final_period": float((wd == wd64).float().mean().item())},
            "paper_reported_s": {"fp32": 20.0, "fp64": 780.0, "cpu_one_core": "> 10800"}}


KURA = {
    "kuramoto_mf": dict(cfg="uniform", coupling=0, scheme=0, steps=100000),
    "kuramoto_mf_em": dict(cfg="uniform", coupling=0, scheme=1, steps=100000),
    "kuramoto_tiled": dict(cfg="uniform", coupling=1, scheme=0, steps=1000),  # a 10^3-step window of 10^5
    "kuramoto_dense_fp32": dict(cfg="dense", coupling=2, scheme=0, steps=20000),
    "kuramoto_dense_bf16x3": dict(cfg="dense", coupling=3, scheme=0, steps=20000),
    "kuramoto_dense_fp16x3": dict(cfg="dense", coupling=4, scheme=0, steps=20000),
}


def kuramoto_cpu_baseline(spec, cfg):
    """The FP64 oracle timed beside a Kuramoto leg on a bounded sample of its
    configuration (a few seconds on the host's threads): the mean field on
    all realizations for 50 steps, the direct all-pairs sum for one
    realization and one step, the dense coupling on realizations 0-7 for 100
    steps."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    N, R = cfg["N"], cfg["R"]
    om = cfg["omega"].astype(np.float64)
    coupling = spec["coupling"]
    if coupling == 0:
        n, rr, kind, Km = 50, R, oracle.MEANFIELD, None
    elif coupling == 1:
        n, rr, kind, Km = 1, 1, oracle.DIRECT, None
    else:
        n, rr, kind, Km = 100, 8, oracle.DENSE, cfg["Kmat"].astype(np.float64)
    t0 = time.perf_counter()
    oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], n, 0, kind, spec["scheme"], cfg["seed"], om,
                              Kmat=Km, r_first=0, r_count=rr, n_threads=threads)
    dt = time.perf_counter() - t0
    sample = f"{rr} realization(s) x N = {N} x {n} step(s), FP64, {dt:.1f} s"
    if coupling == 1:
        stages = 2 if spec["scheme"] == 0 else 1
        return {"value": float(N) * N * rr * n * stages / dt, "unit": "pair terms/s", "cores": threads,
                "kind": "oracle", "sample": sample + " (direct double loop)"}
    return {"value": N * rr * n / dt, "unit": "osc-steps/s", "cores": threads, "kind": "oracle", "sample": sample}


def _circ_err(theta_gpu, phi_ref):
    """Circular phase distance (radians) of GPU revolutions from the oracle's
    unwrapped radians, over max(|phi_ref|, 1)."""
    d = 2 * np.pi * theta_gpu.astype(np.float64) - phi_ref
    d = np.mod(d + np.pi, 2 * np.pi) - np.pi
    return np.abs(d) / np.maximum(np.abs(phi_ref), 1.0)


def kuramoto_parity(spec, cfg, sde, ctx, torch, dev, om, Kt, n=100, reals=(0, 1)):
    """Error against the FP64 oracle in the leg's own launch configuration:
    the GPU integrates all R realizations for the first `n` steps (shared
    noise) and the oracle the listed realizations; the per-oscillator phase
    error is bounded by 1e-5 (1e-4 for the BF16x3 product, whose split keeps
    about 16 bits per term), r(t) samples by 1e-6 (1e-5)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    N, R = cfg["N"], cfg["R"]
    ph = torch.empty((R, N), dtype=torch.float32, device=dev)
    rs = torch.zeros((R, n // 100 + 1), dtype=torch.float64, device=dev)
    desc = sde.sde_kuramoto_desc(N, R, cfg["K"], cfg["D"], cfg["dt"], n, spec["coupling"], 0)
    sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(cfg["seed"], scheme=spec["scheme"], sync=1), ph, om, Kt, rs)
    got, grs = ph.cpu().numpy(), rs.cpu().numpy()
    kind = {0: oracle.MEANFIELD, 1: oracle.MEANFIELD}.get(spec["coupling"], oracle.DENSE)
    Km = cfg["Kmat"].astype(np.float64) if spec["coupling"] >= 2 else None
    tol = 1e-4 if spec["coupling"] == 3 else 1e-5
    worst, rworst = 0.0, 0.0
    t0 = time.perf_counter()
    for r in reals:
        ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], n, 100, kind, spec["scheme"],
                                              cfg["seed"], cfg["omega"].astype(np.float64), Kmat=Km, r_first=r,
                                              r_count=1, n_threads=threads)
        worst = max(worst, float(_circ_err(got[r], ref[0]).max()))
        rworst = max(rworst, float(np.abs(grs[r] - rref[0]).max()))
    return {"against": "FP64 oracle" + (" (Eq. 3 sums)" if spec["coupling"] == 1 else ""),
            "steps": n, "realizations": list(reals), "max_phase_err": worst, "bound": tol,
            "max_abs_diff_r": rworst, "oracle_seconds": time.perf_counter() - t0,
            "ok": bool(worst <= tol and rworst <= 10 * tol)}


def bench_kuramoto(name, args, sde, torch, dev, steps=None, reps=1):
    spec = KURA[name]
    cfg = sde_inputs.kuramoto_uniform() if spec["cfg"] == "uniform" else sde_inputs.kuramoto_dense()
    N, R = cfg["N"], cfg["R"]
    n = steps or spec["steps"]
    om = torch.from_numpy(cfg["omega"]).to(dev)
    Kt = torch.from_numpy(cfg["Kmat"]).to(dev) if spec["coupling"] >= 2 else None
    ph = torch.empty((R, N), dtype=torch.float32, device=dev)
    rs = torch.zeros((R, n // 100 + 1), dtype=torch.float64, device=dev)
    ctx = sde.sde_create(0)
    if getattr(args, "dense_launch", 0) and spec["coupling"] >= 2:
        sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, args.dense_launch)
    desc = sde.sde_kuramoto_desc(N, R, cfg["K"], cfg["D"], cfg["dt"], n, spec["coupling"], 0)
    run = sde.make_run(cfg["seed"], scheme=spec["scheme"])
    stream = torch.cuda.current_stream()
    # warm-up on a short run (kernel load, workspace)
    wdesc = sde.sde_kuramoto_desc(N, R, cfg["K"], cfg["D"], cfg["dt"], min(n, 8), spec["coupling"], 0)
    sde.sde_kuramoto_integrate(ctx, wdesc, run, ph, om, Kt, None)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, Kt, rs)
        e.record(stream)
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e) / 1e3)
    st = sde.sde_get_stats(ctx)
    parity = None if getattr(args, "no_cpu_baseline", True) else kuramoto_parity(spec, cfg, sde, ctx, torch, dev,
                                                                                 om, Kt)
    sde.sde_check(ctx)
    sde.sde_destroy(ctx)
    t = float(np.mean(times))
    osc_steps = N * R * n
    heun = spec["scheme"] == 0
    rec = {"workload": name, "N": N, "R": R, "steps": n, "scheme": "heun" if heun else "euler",
           "seconds": t, "osc_steps_per_s": osc_steps / t,
           "r_final_mean": float(rs.cpu().numpy()[:, -1].mean())}
    if spec["coupling"] == 0:
        ops = mf_ops_per_osc_step(heun)
        rec["roofline"] = {"bound": "alu", "achieved": ops * osc_steps / t / 1e12,
                           "peak": PEAK_FMA_LANES / 1e12, "unit": "T lane-op units/s",
                           "frac": ops * osc_steps / t / PEAK_FMA_LANES, "traffic": None}
        rec["us_per_stage"] = t / (n * (2 if heun else 1)) * 1e6
        rec["oscillators_per_lane"] = st["kura_mf_opt"]
        rec["two_realizations_per_workgroup"] = bool(st["kura_mf_paired"])
        if heun and st["kura_mf_opt"] == 8 and not st["kura_mf_paired"]:
            rec["roofline"]["counters"] = kura_counters("kuramoto_mf")
    elif spec["coupling"] == 1:
        pairs = float(N) * N * R * n * (2 if heun else 1)
        ops = W_FULL + W_TRANS + W_FULL
        rec["pairs_per_s"] = pairs / t
        rec["tile_oscillators_per_lane"] = st["kura_tile"]
        rec["j_slices"] = st["kura_jsplit"]
        rec["roofline"] = {"bound": "alu", "achieved": ops * pairs / t / 1e12, "peak": PEAK_FMA_LANES / 1e12,
                           "unit": "T lane-op units/s", "frac": ops * pairs / t / PEAK_FMA_LANES,
                           "traffic": None, "counters": kura_counters("kuramoto_tiled")}
    else:
        rec["launch"] = {"waves": st["dense_waves"], "xcd_bands": st["dense_xcd_bands"],
                         "kernel": ["k-sliced waves", "two k halves", "row-half waves", "4 waves, K in LDS",
                                    "wave pairs, K in LDS"][st["dense_variant"]]}
        rec["us_per_stage"] = t / (n * (2 if heun else 1)) * 1e6
        gemm_flop = 2.0 * N * N * 2 * R * n * (2 if heun else 1)
        if spec["coupling"] == 2:
            # FP32 MFMA (v_mfma_f32_16x16x4_f32): MI355X's FP32 matrix peak equals its FP32 vector peak
            rec["roofline"] = {"bound": "mfma", "achieved": gemm_flop / t / 1e12, "peak": PEAK_MFMA_FP32 / 1e12,
                               "unit": "TFLOP/s", "frac": gemm_flop / t / PEAK_MFMA_FP32, "traffic": None}
        else:
            executed = 3 * gemm_flop
            rec["gemm_equivalent_tflops"] = gemm_flop / t / 1e12
            rec["roofline"] = {"bound": "mfma", "achieved": executed / t / 1e12, "peak": PEAK_MFMA_16BIT / 1e12,
                               "unit": "TFLOP/s", "frac": executed / t / PEAK_MFMA_16BIT, "traffic": None}
    if not getattr(args, "no_cpu_baseline", True):
        cpu = kuramoto_cpu_baseline(spec, cfg)
        gpu_rate = rec["pairs_per_s"] if spec["coupling"] == 1 else rec["osc_steps_per_s"]
        rec["cpu_baseline"] = dict(cpu, gpu_over_cpu=gpu_rate / cpu["value"])
        rec["parity"] = parity
    return rec


def bench_fig4(args, sde, torch, dev):
    """The globally coupled system of Fig. 4: 2^24 identical oscillators
    (omega = 0), K = 4, D = 1, dt = 0.01, 2000 Heun steps of the mean field
    (Eq. 3) streamed through HBM; r(t) every 100 steps.  Then the same run in
    20 calls of 100 steps, each followed by the phase density P(x; t) in 100
    bins (the figure's time evolution).  The paper's run took about 20 s on
    its GPU: context, not a target."""
    cfg = sde_inputs.kuramoto_fig4(n_steps=args.kura_steps or 2000)
    N, n, M = cfg["N"], cfg["n_steps"], cfg["sample_every"]
    om = torch.zeros(N, dtype=torch.float32, device=dev)
    ph = torch.empty((1, N), dtype=torch.float32, device=dev)
    rs = torch.zeros((1, n // M + 1), dtype=torch.float64, device=dev)
    ctx = sde.sde_create(0)
    desc = sde.sde_kuramoto_desc(N, 1, cfg["K"], cfg["D"], cfg["dt"], n, sde.SDE_MEANFIELD, 0)
    run = sde.make_run(cfg["seed"], sample_every=M)
    stream = torch.cuda.current_stream()
    sde.sde_kuramoto_integrate(ctx, sde.sde_kuramoto_desc(N, 1, cfg["K"], cfg["D"], cfg["dt"], 8,
                                                          sde.SDE_MEANFIELD, 0), run, ph, om, None, None)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(args.steps, 1)):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record(stream)
        sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, None, rs)
        e.record(stream)
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e) / 1e3)
    streamed = sde.sde_get_stats(ctx)["mf_streamed"]
    t = float(np.mean(times))
    single = ph.clone()
    parity = None
    if not getattr(args, "no_cpu_baseline", True):
        # error against the FP64 oracle: one step from the run's final state,
        # every one of the 2^24 oscillators (the oracle's mean-field sums are
        # O(N) per stage, so a step of the full system takes it seconds)
        import oracle
        one = single.clone()
        sde.sde_kuramoto_integrate(ctx, sde.sde_kuramoto_desc(N, 1, cfg["K"], cfg["D"], cfg["dt"], 1,
                                                              sde.SDE_MEANFIELD, 0),
                                   sde.make_run(cfg["seed"], step0=n, init=sde.SDE_INIT_FROM_STATE, sync=1),
                                   one, om, None, None)
        t0 = time.perf_counter()
        ref, _ = oracle.kuramoto_integrate(N, 1, cfg["K"], cfg["D"], cfg["dt"], 1, 0, oracle.MEANFIELD, 0,
                                           cfg["seed"], np.zeros(N), phi0=2 * np.pi * single.cpu().numpy().astype(
                                               np.float64), step0=n,
                                           n_threads=int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count())
        err = _circ_err(one.cpu().numpy()[0], ref[0])
        parity = {"against": "FP64 oracle", "what": f"one Heun step from the state at step {n}, all {N} oscillators",
                  "max_phase_err": float(err.max()), "bound": 1e-5, "oracle_seconds": time.perf_counter() - t0,
                  "ok": bool(err.max() <= 1e-5)}
        del one, ref
    # the time evolution of the phase density, one histogram per 100 steps
    nb = 100
    dens = torch.zeros((n // M + 1, nb + 1), dtype=torch.int64, device=dev)
    chunk = sde.sde_kuramoto_desc(N, 1, cfg["K"], cfg["D"], cfg["dt"], M, sde.SDE_MEANFIELD, 0)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    sde.sde_kuramoto_integrate(ctx, sde.sde_kuramoto_desc(N, 1, cfg["K"], cfg["D"], cfg["dt"], 0,
                                                          sde.SDE_MEANFIELD, 0), run, ph, om, None, None)
    sde.sde_phase_histograms(ctx, ph, nb, dens[0:1])
    for k in range(1, n // M + 1):
        sde.sde_kuramoto_integrate(ctx, chunk, sde.make_run(cfg["seed"], step0=(k - 1) * M,
                                                            init=sde.SDE_INIT_FROM_STATE, sample_every=M),
                                   ph, om, None, None)
        sde.sde_phase_histograms(ctx, ph, nb, dens[k:k + 1])
    e.record(stream)
    torch.cuda.synchronize()
    t_snap = s.elapsed_time(e) / 1e3
    sde.sde_check(ctx)
    sde.sde_destroy(ctx)
    h = dens.cpu().numpy()[:, :nb] * nb / N
    r = rs.cpu().numpy()[0]
    osc_steps = float(N) * n
    ops, byts = mfs_ops_per_osc_step(True), mfs_bytes_per_osc_step(True)
    hbm = byts * osc_steps / t
    alu = ops * osc_steps / t
    traffic = (FIG4_TRAFFIC_PER_OSC_STEP * osc_steps
               if _source_sha1("kuramoto.hip", "device_common.h") == FIG4_TRAFFIC_SOURCE_SHA1 else None)
    return {"workload": "kuramoto_fig4", "N": N, "R": 1, "omega": 0.0, "K": cfg["K"], "D": cfg["D"],
            "dt": cfg["dt"], "steps": n, "scheme": "heun", "streamed_through_hbm": bool(streamed),
            "seconds": t, "osc_steps_per_s": osc_steps / t, "us_per_step": t / n * 1e6,
            "roofline": {"bound": "hbm", "achieved": hbm / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                         "frac": hbm / PEAK_HBM, "traffic": traffic, "bytes_per_osc_step": byts},
            "alu": {"achieved": alu / 1e12, "peak": PEAK_FMA_LANES / 1e12, "frac": alu / PEAK_FMA_LANES,
                    "ops_per_osc_step": ops},
            "r_t": [round(float(x), 5) for x in r],
            "r_self_consistency": 0.8314620247541972,
            "r_late_minus_self_consistency": float(r[-10:].mean() - 0.8314620247541972),
            "parity": parity,
            "density_snapshots": {"every_steps": M, "bins": nb, "seconds_with_snapshots": t_snap,
                                  "same_as_single_call": bool(torch.equal(single, ph)),
                                  "peak_density_at_t": {str(k * M * cfg["dt"]): round(float(h[k].max()), 4)
                                                        for k in sorted({0, 5, 10, 15, n // M}) if k <= n // M}},
            "paper_reported_s": 20.0}


def _timed(torch, fn):
    stream = torch.cuda.current_stream()
    fn()  # warm-up: code object, workspace, tuning, graph
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record(stream)
    fn()
    e.record(stream)
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3


def bench_sweep(args, sde, torch, dev):
    """Throughput against the number of particles N (Fig. 5), each kernel
    with and without the small-N remedy of Sec. 6: JJ paths of one point
    (remedy: many parameter points at once, 2^20 paths in all), the
    all-pairs sum for one realization (remedy: j split over workgroups), the
    mean field for one realization (remedy: 16 realizations per launch), the
    dense BF16x3 product at 256 realizations (remedy: N R = 2^20 per launch).
    GFLOPS use the paper's operation counts per particle-step: 79 (JJ),
    44 + 6 N (all pairs), 66 (mean field)."""
    ctx = sde.sde_create(0)
    out = {"paper_saturation_gflops": {"jj": 450, "kuramoto_mf": 106}}
    rows = []
    for lg in range(8, 23, 2):
        P, n = 1 << lg, 20000
        pt = sde_inputs.jj_point(n_paths=P, n_steps=n)
        st = tuple(torch.empty(P, dtype=dt, device=dev)
                   for dt in (torch.float32, torch.int32, torch.float32, torch.float64))
        run = sde.make_run(sde_inputs.seed_of(30))
        t = _timed(torch, lambda: sde.sde_jj_integrate(ctx, [pt], run, *st))
        ppt = sde.sde_get_stats(ctx)["jj_paths_per_lane"]
        rec = {"N": P, "seconds": t, "path_steps_per_s": P * n / t, "paper_gflops": 79 * P * n / t / 1e9,
               "paths_per_lane": ppt}
        if P < (1 << 20):
            q = (1 << 20) // P  # the same paths per point, many points
            pts = [dict(pt, f=0.5 * k / q) for k in range(q)]
            stb = tuple(torch.empty(1 << 20, dtype=dt, device=dev)
                        for dt in (torch.float32, torch.int32, torch.float32, torch.float64))
            tb = _timed(torch, lambda: sde.sde_jj_integrate(ctx, pts, run, *stb))
            rec["batched"] = {"points": q, "path_steps_per_s": (1 << 20) * n / tb,
                              "paper_gflops": 79 * (1 << 20) * n / tb / 1e9}
        rows.append(rec)
        print(f"sweep jj N={P}: {rec['path_steps_per_s']:.3g} path-steps/s", file=sys.stderr, flush=True)
    out["jj"] = rows

    def kura(N, R, n, coupling, jsplit=0):
        cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
        om = torch.from_numpy(cfg["omega"]).to(dev)
        ph = torch.empty((R, N), dtype=torch.float32, device=dev)
        sde.sde_set_option(ctx, sde.SDE_OPT_KURA_JSPLIT, jsplit)
        desc = sde.sde_kuramoto_desc(N, R, cfg["K"], cfg["D"], cfg["dt"], n, coupling, 0)
        run = sde.make_run(cfg["seed"])
        t = _timed(torch, lambda: sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, None, None))
        return t, sde.sde_get_stats(ctx)

    rows = []
    for N in (256, 1024, 4096, 16384, 65536):
        n = 20 if N >= 16384 else 200
        t1, _ = kura(N, 1, n, sde.SDE_TILED, jsplit=1)
        tj, stj = kura(N, 1, n, sde.SDE_TILED, jsplit=0)
        ops = (44 + 6 * N) * N * n
        rows.append({"N": N, "steps": n, "pairs_per_s": 2.0 * N * N * n / t1, "paper_gflops": ops / t1 / 1e9,
                     "j_split": {"J": stj["kura_jsplit"], "pairs_per_s": 2.0 * N * N * n / tj,
                                 "paper_gflops": ops / tj / 1e9}})
        print(f"sweep tiled N={N}: J=1 {rows[-1]['pairs_per_s']:.3g}, J={stj['kura_jsplit']} "
              f"{rows[-1]['j_split']['pairs_per_s']:.3g} pairs/s", file=sys.stderr, flush=True)
    out["kuramoto_all_pairs"] = rows
    rows = []
    for lg in range(10, 25, 2):
        N, n = 1 << lg, 1000
        t1, st1 = kura(N, 1, n, sde.SDE_MEANFIELD)
        rec = {"N": N, "steps": n, "osc_steps_per_s": N * n / t1, "paper_gflops": 66 * N * n / t1 / 1e9,
               "streamed": st1["mf_streamed"]}
        if N <= (1 << 20):
            t16, _ = kura(N, 16, n, sde.SDE_MEANFIELD)
            rec["16_realizations"] = {"osc_steps_per_s": 16 * N * n / t16, "paper_gflops": 66 * 16 * N * n / t16 / 1e9}
        rows.append(rec)
        print(f"sweep mean field N={N}: {rec['osc_steps_per_s']:.3g} osc-steps/s", file=sys.stderr, flush=True)
    out["kuramoto_mean_field"] = rows
    # dense K_ij, BF16x3 product, 256 realizations; remedy for small N: more
    # realizations per launch (N R = 2^20, the benchmark's product width)
    rows = []
    for N in (512, 1024, 2048, 4096, 8192):
        n = 200 if N <= 4096 else 50
        Kt = torch.from_numpy(sde_inputs.dense_coupling(N, 4.0, sde_inputs.seed_of(31))).to(dev)
        om = torch.from_numpy(sde_inputs.kuramoto_omega(N, 0.5, sde_inputs.seed_of(32))).to(dev)
        rec = {"N": N, "steps": n}
        for key, R in (("R256", 256), ("filled", max(256, (1 << 20) // N))):
            if key == "filled" and R == 256:
                continue
            ph = torch.empty((R, N), dtype=torch.float32, device=dev)
            desc = sde.sde_kuramoto_desc(N, R, 4.0, 0.05, 0.005, n, sde.SDE_DENSE_BF16X3, 0)
            run = sde.make_run(sde_inputs.seed_of(33))
            t = _timed(torch, lambda: sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, Kt, None))
            executed = 3 * 2.0 * N * N * 2 * R * n * 2
            rec[key] = {"R": R, "osc_steps_per_s": N * R * n / t, "us_per_stage": t / (2 * n) * 1e6,
                        "mfma_frac": executed / t / PEAK_MFMA_16BIT}
            del ph
        rows.append(rec)
        print(f"sweep dense N={N}: R=256 {rec['R256']['osc_steps_per_s']:.3g} osc-steps/s "
              f"({100 * rec['R256']['mfma_frac']:.1f} % MFMA)", file=sys.stderr, flush=True)
        del Kt
    out["kuramoto_dense_bf16x3"] = rows
    sde.sde_check(ctx)
    sde.sde_destroy(ctx)
    return {"workload": "sweep", "sweep": out}


# Instruction forms of the issue-cost probe (paper_0903_3852_amd/probe/valu_issue.hip), in its mode order.
VALU_FORMS = ["v_add_f32 v,v", "v_add_f32 v,s", "v_fma_f32 v,v,v", "v_fma_f32 s,v,v", "v_mul_f32 v,v",
              "v_xor_b32 v,v", "v_xor_b32 v,s", "v_add_u32 v,v", "v_lshrrev_b32 8,v", "v_mad_u64_u32 v,s,v",
              "v_mul_hi_u32 v,v", "v_cvt_f32_u32", "v_floor_f32", "v_add_f64", "v_fma_f64", "v_cvt_f64_f32",
              "v_sin_f32", "v_cos_f32", "v_log_f32", "v_sqrt_f32", "v_mov_b32_dpp row_shr", "v_mov_b32 v",
              "v_add_f32 v,const", "v_fma_f32 v,const,const", "v_mul_f32 const,v", "v_xor_b32 const,v",
              "v_add_u32 const,v"]


def bench_valu_costs(args):
    """Issue cost of single VALU instruction forms (SIMD cycles per wave64
    instruction at 8 waves per SIMD, 8 independent chains per lane, at the
    2.4 GHz peak clock): the cost model behind the ALU rooflines."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_0903_3852_amd", "libvaluprobe.so"))
    lib.valu_issue_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    lib.valu_issue_time.restype = ctypes.c_int
    assert lib.valu_issue_modes() == len(VALU_FORMS)
    iters = 20000
    out = {}
    for mode, name in enumerate(VALU_FORMS):
        ms = ctypes.c_float()
        if lib.valu_issue_time(mode, iters, ctypes.byref(ms)) != 0:
            raise RuntimeError(f"valu probe mode {mode} failed")
        instr = 2048 * 4.0 * iters * 8.0
        out[name] = round(1024 * 2.4e9 * ms.value * 1e-3 / instr, 3)
    # Sustained matrix-core rate of the MFMA forms of the dense coupling, at
    # 1, 2 and 8 waves per SIMD (256, 512, 2048 workgroups of 4 waves), in
    # TFLOP/s and in SIMD cycles per MFMA at 2.4 GHz
    lib.mfma_rate_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
    lib.mfma_rate_time.restype = ctypes.c_int
    mfma = {}
    for form, (name, flop, peak) in enumerate([("v_mfma_f32_16x16x32_bf16", 16384, PEAK_MFMA_16BIT),
                                               ("v_mfma_f32_16x16x32_f16", 16384, PEAK_MFMA_16BIT),
                                               ("v_mfma_f32_16x16x4_f32", 2048, PEAK_MFMA_FP32)]):
        rows = {}
        for waves, blocks in ((1, 256), (2, 512), (8, 2048)):
            it = 4000 if form < 2 else 8000
            ms = ctypes.c_float()
            if lib.mfma_rate_time(form, blocks, it, ctypes.byref(ms)) != 0:
                raise RuntimeError(f"mfma probe form {form} failed")
            n = blocks * 4.0 * it * 8.0
            rate = n * flop / (ms.value * 1e-3)
            rows[f"{waves}_waves_per_simd"] = {"tflops": round(rate / 1e12, 1), "frac_of_peak": round(rate / peak, 3),
                                               "cycles_per_mfma": round(1024 * 2.4e9 * ms.value * 1e-3 / n, 2)}
        mfma[name] = rows
    # The same bf16 MFMA fed from memory as the dense coupling feeds it: per 96
    # MFMAs a wave loads 24 (16, 8) 1 KB fragments one iteration ahead, 2 waves
    # per SIMD, from a 2 MiB (L2-resident) or 1 GiB buffer
    lib.mfma_feed_time.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_longlong,
                                   ctypes.POINTER(ctypes.c_float)]
    lib.mfma_feed_time.restype = ctypes.c_int
    feed = {}
    for loads in (24, 16, 8):
        for label, nbytes in (("l2", 2 << 20), ("hbm", 1 << 30)):
            it, blocks = 1000, 256
            ms = ctypes.c_float()
            if lib.mfma_feed_time(loads, blocks, it, nbytes, ctypes.byref(ms)) != 0:
                raise RuntimeError(f"mfma feed probe ({loads} loads) failed")
            t = ms.value * 1e-3
            n = blocks * 8.0 * it * 96
            feed[f"{loads}_loads_per_96_mfma_{label}"] = {
                "tflops": round(n * 16384 / t / 1e12, 1), "frac_of_peak": round(n * 16384 / t / PEAK_MFMA_16BIT, 3),
                "bytes_per_clk_per_cu": round(blocks * 8.0 * it * loads * 1024 / t / 256 / 2.4e9, 1)}
    rec = {"workload": "valu_costs", "unit": "SIMD cycles per wave64 instruction", "cycles": out,
           "mfma_rate": mfma, "mfma_fed_from_memory": feed}
    if getattr(args, "mfma_sustained", False):
        # the bf16 cases of the dense coupling over 20-80 ms launches (clock under sustained matrix load)
        ms = ctypes.c_float()
        if lib.mfma_rate_time(0, 512, 200000, ctypes.byref(ms)) != 0:
            raise RuntimeError("mfma probe failed")
        reg = 512 * 4.0 * 200000 * 8 * 16384 / (ms.value * 1e-3)
        if lib.mfma_feed_time(24, 256, 50000, 2 << 20, ctypes.byref(ms)) != 0:
            raise RuntimeError("mfma feed probe failed")
        fed = 256 * 8.0 * 50000 * 96 * 16384 / (ms.value * 1e-3)
        rec["mfma_sustained"] = {"register_only_2_waves_tflops": round(reg / 1e12, 1),
                                 "fed_24_loads_l2_tflops": round(fed / 1e12, 1),
                                 "fed_frac_of_peak": round(fed / PEAK_MFMA_16BIT, 3)}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="jj_scan",
                    choices=["jj_scan", "jj_batch", "jj_surrogate", "jj_surrogate_anm", "jj_fig2", "kuramoto_fig4",
                             "sweep", "valu_costs"] + sorted(KURA))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kuramoto", action="store_true")
    ap.add_argument("--dense-launch", type=int, default=0,
                    help="kuramoto_dense_*: force a dense launch choice (1-10, as SDE_OPT_DENSE_LAUNCH; 0 tunes)")
    ap.add_argument("--mfma-sustained", action="store_true",
                    help="valu_costs: also time the dense coupling's bf16 MFMA cases over 20-80 ms launches")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--model-steps", type=int, default=200000,
                    help="Heun steps per path (the workload uses 2e5; smaller only for profiling)")
    ap.add_argument("--kura-steps", type=int, default=None,
                    help="steps of a kuramoto_* workload (default: its own; fewer only for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the library has no "
              "multi-GPU launch.  The JJ scan would shard by points across GPUs with no exchange but a "
              "final gather of the per-point sums.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_0903_3852_amd as sde

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "jj_scan":
        out = bench_jj(args, sde, torch, dev)
        progress("jj_scan leg done")
        if not args.no_kuramoto:
            out["kuramoto"] = []
            for w in ("kuramoto_mf", "kuramoto_mf_em", "kuramoto_tiled", "kuramoto_dense_bf16x3",
                      "kuramoto_dense_fp16x3", "kuramoto_dense_fp32"):
                out["kuramoto"].append(bench_kuramoto(w, args, sde, torch, dev))
                progress(f"{w} leg done")
            jb = bench_jj_batch(args, sde, torch, dev)
            jb["tail_efficiency"] = jb["path_steps_per_s"] / (out["config"]["path_steps_per_step"] /
                                                            (out["kernel_ms"] / 1e3))
            out["jj_batch"] = jb
            progress("jj_batch leg done")
            out["surrogate"] = bench_surrogate(args, sde, torch, dev)
            out["surrogate_anm"] = bench_surrogate(args, sde, torch, dev, variant="anm")
            out["fig2"] = bench_fig2(args, sde, torch, dev)
            progress("jj_fig2 leg done")
            out["fig4"] = bench_fig4(args, sde, torch, dev)
            progress("kuramoto_fig4 leg done")
    elif args.workload == "jj_batch":
        out = bench_jj_batch(args, sde, torch, dev)
    elif args.workload == "jj_surrogate":
        out = bench_surrogate(args, sde, torch, dev)
    elif args.workload == "jj_surrogate_anm":
        out = bench_surrogate(args, sde, torch, dev, variant="anm")
    elif args.workload == "jj_fig2":
        out = bench_fig2(args, sde, torch, dev)
    elif args.workload == "kuramoto_fig4":
        out = bench_fig4(args, sde, torch, dev)
    elif args.workload == "sweep":
        out = bench_sweep(args, sde, torch, dev)
    elif args.workload == "valu_costs":
        out = bench_valu_costs(args)
    else:
        out = bench_kuramoto(args.workload, args, sde, torch, dev, steps=args.kura_steps, reps=args.steps)
    if args.calibrate_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = 1 << 30
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
