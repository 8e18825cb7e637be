"""The launch layer on the GPU: autotuned paths-per-lane choices, the tune
cache, recorded HIP graphs, and one persistent launch over an uneven batch of
points (different path and step counts), all through the C ABI.

The per-path arithmetic does not depend on how paths are grouped into
lanes or on whether launches are replayed from a graph, so those results
must be bitwise identical; the uneven batch is compared with the oracle
(paired per-point time averages within 3 SE + 1e-4).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import sde_inputs

pytestmark = pytest.mark.gpu


def _state(n, dev):
    return (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float64, device=dev))


def _jj(sde, ctx, dev, pts, seed=21):
    n = sum(p["n_paths"] for p in pts)
    st = _state(n, dev)
    ps = torch.empty((len(pts), 2), dtype=torch.float64, device=dev)
    sde.sde_jj_integrate(ctx, pts, sde.make_run(seed, sync=1), *st, ps)
    return [x.clone() for x in st] + [ps.clone()]


def _points():
    return [sde_inputs.jj_point(f=0.03 * i, D=10 ** (-3 + 0.2 * i), n_paths=100 + 97 * i,
                                n_steps=300 + 41 * i, n_transient=100) for i in range(7)]


def test_paths_per_lane_bit_identical(gpu):
    sde, _, dev = gpu
    ctx = sde.sde_create(0)
    try:
        outs = []
        for ppt in (1, 2, 4):
            sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, ppt)
            outs.append(_jj(sde, ctx, dev, _points()))
            assert sde.sde_get_stats(ctx)["jj_paths_per_lane"] == ppt
        for o in outs[1:]:
            # per-path state is bitwise identical; the point sums group the
            # paths into chunks of 64 x (paths per lane), so they agree to
            # rounding only
            for a, b in zip(outs[0][:4], o[:4]):
                assert torch.equal(a, b)
            torch.testing.assert_close(outs[0][4], o[4], rtol=1e-12, atol=1e-12)
    finally:
        sde.sde_destroy(ctx)


def test_autotuner_and_cache(gpu, tmp_path):
    sde, _, dev = gpu
    cache = tmp_path / "tune.json"
    ctx = sde.sde_create(0)
    try:
        sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 2)
        ref = _jj(sde, ctx, dev, _points())
        sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 0)
        sde.sde_set_tune_cache(ctx, str(cache))
        got = _jj(sde, ctx, dev, _points())
        st = sde.sde_get_stats(ctx)
        assert st["tuned"] == 1 and st["jj_paths_per_lane"] in (1, 2, 4)
        for a, b in zip(ref[:4], got[:4]):
            assert torch.equal(a, b)
        torch.testing.assert_close(ref[4], got[4], rtol=1e-12, atol=1e-12)
        saved = json.loads(cache.read_text())
        assert any(k.startswith("jj|gfx950") for k in saved)
        # same shape class: no second tuning, and the launch sequence replays
        _jj(sde, ctx, dev, _points())
        st2 = sde.sde_get_stats(ctx)
        assert st2["tuned"] == 0
    finally:
        sde.sde_destroy(ctx)
    # a new context reads the choice from the file
    ctx = sde.sde_create(0)
    try:
        sde.sde_set_tune_cache(ctx, str(cache))
        _jj(sde, ctx, dev, _points())
        assert sde.sde_get_stats(ctx)["tuned"] == 0
    finally:
        sde.sde_destroy(ctx)


def test_graph_replay_matches_eager(gpu):
    """Replays of a recorded call, with unrelated eager work and
    synchronizations between them, each equal the eager launch."""
    sde, _, dev = gpu
    ctx = sde.sde_create(0)
    try:
        pts = _points()
        n = sum(p["n_paths"] for p in pts)
        st = _state(n, dev)
        ps = torch.empty((len(pts), 2), dtype=torch.float64, device=dev)
        run = sde.make_run(5, sync=1)
        sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, 0)
        sde.sde_jj_integrate(ctx, pts, run, *st, ps)
        eager = [x.clone() for x in st] + [ps.clone()]
        sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, 1)
        replayed = 0
        for rep in range(4):
            for x in st:
                x.zero_()
            junk = torch.randn(1 << 20, device=dev).sum()  # eager work between replays
            torch.cuda.synchronize()
            sde.sde_jj_integrate(ctx, pts, run, *st, ps)
            replayed += sde.sde_get_stats(ctx)["graph_replayed"]
            for a, b in zip(eager, list(st) + [ps]):
                assert torch.equal(a, b), rep
            del junk
        assert replayed >= 3
    finally:
        sde.sde_destroy(ctx)


def test_graph_keys_distinguish_variants(gpu):
    """Same buffers and sizes, different product variant: each call must run
    its own kernels, not a graph recorded for another variant."""
    sde, _, dev = gpu
    N, R, n = 256, 32, 20
    omega = torch.from_numpy(sde_inputs.kuramoto_omega(N, 0.5, 2)).to(dev)
    K = torch.from_numpy(sde_inputs.dense_coupling(N, 4.0, 2)).to(dev)
    ctx = sde.sde_create(0)
    try:
        res = {}
        for graphs in (0, 1):
            sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, graphs)
            ph = torch.empty((R, N), dtype=torch.float32, device=dev)
            for coupling in (2, 3, 4, 3, 2):
                desc = sde.sde_kuramoto_desc(N, R, 4.0, 0.05, 0.005, n, coupling, 0)
                sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(1, sync=1), ph, omega, K)
                res.setdefault((graphs, coupling), []).append(ph.clone())
        for (g, c), outs in res.items():
            for o in outs:
                assert torch.equal(o, res[(0, c)][0]), (g, c)
    finally:
        sde.sde_destroy(ctx)


@pytest.mark.parametrize("coupling", [1, 3])
def test_kuramoto_chunk_graphs_match_eager(gpu, coupling):
    """Tiled and dense step loops recorded in chunks of steps (device-side
    step counter) equal direct launches, over repeated calls."""
    sde, _, dev = gpu
    N, R, n, M = 600, 40, 237, 50
    omega = torch.from_numpy(sde_inputs.kuramoto_omega(N, 1.0, 1)).to(dev)
    K = torch.from_numpy(sde_inputs.dense_coupling(N, 3.0, 1)).to(dev) if coupling >= 2 else None
    desc = sde.sde_kuramoto_desc(N, R, 3.0, 0.1, 0.01, n, coupling, 0)
    ctx = sde.sde_create(0)
    try:
        outs = []
        for graphs in (0, 1, 1, 1):
            sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, graphs)
            ph = torch.empty((R, N), dtype=torch.float32, device=dev)
            rs = torch.zeros((R, n // M + 1), dtype=torch.float64, device=dev)
            sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(3, sample_every=M, sync=1), ph, omega, K, rs)
            outs.append((ph, rs))
            torch.randn(1000, device=dev).sum().item()
        for ph, rs in outs[1:]:
            assert torch.equal(outs[0][0], ph)
            assert torch.equal(outs[0][1], rs)
        assert torch.all(outs[0][1] > 0)
    finally:
        sde.sde_destroy(ctx)


def test_uneven_batch_matches_oracle(gpu):
    """One persistent launch over 96 random points of the batch distribution
    (a, omega, f, log10 D, gamma) with path counts in [1, 600] and step
    counts in [200, 6000] (transient: half)."""
    sde, ctx, dev = gpu
    pts = sde_inputs.jj_batch(n_points=96, seed=77, path_range=(1, 600), step_range=(200, 6000))
    seed = sde_inputs.seed_of(5)
    out = _jj(sde, ctx, dev, pts, seed=seed)
    assert sde.sde_get_stats(ctx)["work_items"] >= 96
    ref = oracle.jj_integrate(pts, seed)
    acc = out[3].cpu().numpy()
    off = 0
    worst = 0.0
    for p in pts:
        n = p["n_paths"]
        W = p["n_steps"] - p["n_transient"]
        g, r = acc[off:off + n] / W, ref["acc"][off:off + n] / W
        d = g - r
        se = d.std(ddof=1) / np.sqrt(n) if n > 1 else 0.0
        worst = max(worst, abs(d.mean()) / (3 * se + 1e-4))
        off += n
    print(f"uneven batch: worst |mean diff| / (3 SE + 1e-4) = {worst:.3f}")
    assert worst <= 1.0
    sums = out[4].cpu().numpy()
    np.testing.assert_allclose(sums[:, 0], [acc[o:o + p["n_paths"]].sum() / (p["n_steps"] - p["n_transient"])
                                            for o, p in zip(np.cumsum([0] + [q["n_paths"] for q in pts])[:-1], pts)],
                               rtol=1e-12)


def test_uneven_batch_full_size_sampled(gpu):
    """The full uneven batch -- 2048 points with 256-8192 paths and
    5*10^4-4*10^5 steps (half transient), one persistent launch as the
    benchmark runs it -- checked on sampled points: the longest and shortest
    runs, the most and fewest paths, and two more; the oracle integrates the
    first 48 paths of each under its batch index and the time-averaged
    velocities are compared pairwise.  Every point's sums equal the sums of
    its per-path accumulators."""
    sde, ctx, dev = gpu
    pts = sde_inputs.jj_batch()
    seed = sde_inputs.seed_of(5)
    paths = np.array([p["n_paths"] for p in pts])
    steps = np.array([p["n_steps"] for p in pts])
    first = np.concatenate([[0], np.cumsum(paths)[:-1]])
    n = int(paths.sum())
    print(f"uneven batch full size: {len(pts)} points, {n} paths, {int((paths * steps).sum())} path-steps",
          flush=True)
    acc = torch.empty(n, dtype=torch.float64, device=dev)
    ps = torch.empty((len(pts), 2), dtype=torch.float64, device=dev)
    sde.sde_jj_integrate(ctx, pts, sde.make_run(seed, sync=1), None, None, None, acc, ps)
    sums = ps.cpu().numpy()
    a = acc.cpu().numpy()
    W = steps - steps // 2
    assert np.all(np.isfinite(sums)) and np.all(np.abs(sums[:, 0] / paths) < 10.0)
    qs = sorted({int(np.argmax(steps)), int(np.argmin(steps)), int(np.argmax(paths)), int(np.argmin(paths)),
                 777, 2047})
    sub = [dict(pts[q], n_paths=48) for q in qs]
    ref = oracle.jj_integrate(sub, seed, point_ids=qs)
    for i, q in enumerate(qs):
        g = a[first[q]:first[q] + 48] / W[q]
        r = ref["acc"][48 * i:48 * (i + 1)] / W[q]
        d = g - r
        se = d.std(ddof=1) / np.sqrt(d.size)
        print(f"batch point {q} ({paths[q]} paths, {steps[q]} steps): gpu {g.mean():.6f} oracle {r.mean():.6f} "
              f"diff {d.mean():.2e} SE {se:.2e}")
        assert abs(d.mean()) <= 3 * se + 1e-4, q
    vb = [a[f:f + p].sum() / w for f, p, w in zip(first, paths, W)]
    np.testing.assert_allclose(sums[:, 0], vb, rtol=1e-12, atol=1e-12)


def test_options_validation(gpu):
    sde, ctx, dev = gpu
    for opt, val in [(sde.SDE_OPT_AUTOTUNE, 2), (sde.SDE_OPT_GRAPHS, -1), (sde.SDE_OPT_JJ_PPT, 3), (99, 0)]:
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, opt, val)
