"""sde_jj_integrate_noalloc, the entry point that allocates nothing, against
sde_jj_integrate on the same inputs.

Both run the same kernels over the same work items (the paths per lane are
forced equal), so every output -- theta, winding, v, the window sums and
the per-point sums -- must agree bit for bit.  The no-allocation variant
keeps its tables in one static device array that every call reuses: two
calls in a row, the second smaller than the first (fewer points, chunks and
drive tables, a nonzero start step), show that what the first call left in
the array does not leak into the second.  A call that needs more scratch
than the array holds fails on the host before anything is launched.
"""
import numpy as np
import pytest
import torch

import paper_0903_3852_amd as sde_mod
import sde_inputs

pytestmark = pytest.mark.gpu


def _outputs(n_paths, n_pts, dev, fill=0):
    return [torch.full((n_paths,), fill, dtype=torch.float32, device=dev),
            torch.full((n_paths,), fill, dtype=torch.int32, device=dev),
            torch.full((n_paths,), fill, dtype=torch.float32, device=dev),
            torch.full((n_paths,), fill, dtype=torch.float64, device=dev),
            torch.full((n_pts, 2), fill, dtype=torch.float64, device=dev)]


def _batch(rng, n_pts, max_paths, max_steps):
    """Points of every kind (inertial / overdamped, both potentials), ragged
    path counts, uneven lengths, windows starting inside the call, several
    drive periods (distinct drive tables)."""
    pts = []
    for q in range(n_pts):
        n_steps = int(rng.integers(max_steps // 4, max_steps + 1))
        pts.append(sde_inputs.jj_point(
            m=float(rng.choice([1.0, 0.0])), gamma=float(rng.uniform(0.5, 1.5)), a=float(rng.uniform(2, 6)),
            omega=float(rng.uniform(3, 7)), f=float(rng.uniform(0, 0.5)), D=float(10 ** rng.uniform(-4, -1)),
            n_paths=int(rng.integers(1, max_paths + 1)), steps_per_period=int(rng.choice([100, 200, 333])),
            n_steps=n_steps, n_transient=int(rng.integers(0, n_steps)), potential=int(rng.integers(0, 2))))
    return pts


def test_noalloc_matches_the_allocating_entry_point(gpu):
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 2)
    rng = np.random.default_rng(20260)
    calls = [(_batch(rng, 40, 700, 900), 0), (_batch(rng, 7, 150, 300), 8)]
    for k, (pts, step0) in enumerate(calls):
        n = sum(p["n_paths"] for p in pts)
        print(f"noalloc call {k}: {len(pts)} points, {n} paths, step0 {step0}", flush=True)
        run = sde.make_run(77 + k, step0=step0, sync=1)
        ref = _outputs(n, len(pts), dev)
        sde.sde_jj_integrate(ctx, pts, run, *ref)
        got = _outputs(n, len(pts), dev, fill=-3)
        sde.sde_jj_integrate_noalloc(ctx, pts, run, *got)
        torch.cuda.synchronize()
        for name, a, b in zip(("theta", "winding", "v", "acc", "point_sums"), got, ref):
            assert torch.equal(a, b), (k, name)
        assert bool(torch.isfinite(got[0]).all()) and bool(got[4].abs().sum() > 0)


def test_noalloc_resumes_like_one_call(gpu):
    """FROM_STATE through the no-allocation entry point: a run split at a
    multiple of 4 and of M equals one run bit for bit."""
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 2)
    pts = [sde_inputs.jj_point(n_paths=300, n_steps=800, n_transient=100, D=0.01),
           sde_inputs.jj_point(m=0.0, f=1.3, n_paths=65, n_steps=800, n_transient=0, D=0.01, potential=1)]
    n = 365
    whole = _outputs(n, 2, dev)
    sde.sde_jj_integrate_noalloc(ctx, pts, sde.make_run(5, sync=1), *whole)
    part = _outputs(n, 2, dev)
    sde.sde_jj_integrate_noalloc(ctx, [dict(p, n_steps=400) for p in pts], sde.make_run(5, sync=1), *part)
    sde.sde_jj_integrate_noalloc(ctx, [dict(p, n_steps=400) for p in pts],
                                 sde.make_run(5, step0=400, init=sde.SDE_INIT_FROM_STATE, sync=1), *part)
    for a, b in zip(part, whole):
        assert torch.equal(a, b)


def test_noalloc_rejects_a_call_beyond_its_scratch(gpu):
    """100000 one-path points need 100000 x (96 + 24) B > 8 MiB: an error on
    the host, the outputs untouched."""
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 2)
    pts = sde.make_points([sde_inputs.jj_point(n_paths=1, n_steps=4)] * 100000)
    out = _outputs(100000, 100000, dev, fill=-9)
    with pytest.raises(sde_mod.SDEError) as e:
        sde.sde_jj_integrate_noalloc(ctx, pts, sde.make_run(1, sync=1), *out)
    assert e.value.status == sde.SDE_ERR_INVALID
    assert "maximum" in sde.sde_last_error(ctx)
    torch.cuda.synchronize()
    for t in out:
        assert bool((t == -9).all())
    # the context still works afterwards
    small = _outputs(64, 1, dev)
    sde.sde_jj_integrate_noalloc(ctx, [sde_inputs.jj_point(n_paths=64, n_steps=40)], sde.make_run(1, sync=1), *small)
