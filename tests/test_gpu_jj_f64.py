"""GPU parity of the double-precision Josephson-junction path
(sde_jj_integrate_f64) against the FP64 oracle, and the single- against
double-precision comparison of the paper's precision study (Sec. 5, Fig. 2).

Tolerances (relative, |d| / max(|ref|, 1)):
  * per path, 100 steps of the -sin(phi) form at 400 steps per period:
    1e-11 -- both sides are FP64; they differ in the rounding of libm and
    GPU math functions (about one ulp), in fused multiply-adds, and in that
    the GPU keeps the phase as a wrapped fraction plus a winding count;
  * the paper's potential, where barrier tops amplify rounding (~10^3 over
    100 steps at dt = 0.01 period): one step from the oracle's state 1e-13,
    100-step trajectories 1e-10;
  * ensembles: paired |gpu - oracle| <= 3 SE + 1e-4; SP against DP
    histograms: two-sample chi-square p > 1e-4 (the paper's statement that
    they differ only within the statistical error).
"""
import numpy as np
import pytest
import torch
from scipy import stats

import oracle
import sde_inputs
from conftest import rel_err

pytestmark = pytest.mark.gpu
P2 = sde_inputs.POT_SIN2PI


def _state(n, dev, dt=torch.float64):
    return (torch.empty(n, dtype=dt, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=dt, device=dev), torch.empty(n, dtype=torch.float64, device=dev))


def _run64(gpu, pts, seed, step0=0, scheme=0, state=None, sums=True):
    sde, ctx, dev = gpu
    n = sum(p["n_paths"] for p in pts)
    init = sde.SDE_INIT_FROM_STATE if state is not None else sde.SDE_INIT_PHILOX
    st = state if state is not None else _state(n, dev)
    ps = torch.zeros((len(pts), 2), dtype=torch.float64, device=dev) if sums else None
    sde.sde_jj_integrate_f64(ctx, pts, sde.make_run(seed, step0=step0, scheme=scheme, init=init, sync=1), *st, ps)
    return st, ps


def _coord(st, period):
    return period * (st[0].cpu().numpy() + st[1].cpu().numpy().astype(np.float64))


def test_f64_per_path_100_steps(gpu):
    pts = sde_inputs.jj_single(n_paths=4096, n_steps=100)
    seed = sde_inputs.seed_of(1)
    st, _ = _run64(gpu, pts, seed, sums=False)
    ref = oracle.jj_integrate(pts, seed)
    e = max(rel_err(_coord(st, 2 * np.pi), ref["phi"]).max(), rel_err(st[2].cpu().numpy(), ref["v"]).max())
    print(f"FP64 per-path relative error over 100 steps: {e:.2e}")
    assert e <= 1e-11


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("m", [1.0, 0.0])
def test_f64_schemes_and_potentials(gpu, scheme, m):
    """Both potentials, inertial and overdamped, Heun and Euler, 60 steps."""
    for pot, period, tol in [(0, 2 * np.pi, 1e-11), (P2, 1.0, 1e-10)]:
        pt = sde_inputs.jj_point(m=m, gamma=0.9 if m else 1.3, f=0.3 if m else (1.2 if pot == 0 else 7.0), D=0.01,
                                 n_paths=1000, steps_per_period=200, n_steps=60, potential=pot)
        st, _ = _run64(gpu, [pt], 5, scheme=scheme, sums=False)
        ref = oracle.jj_integrate([pt], 5, scheme=scheme)
        e = max(rel_err(_coord(st, period), ref["phi"]).max(), rel_err(st[2].cpu().numpy(), ref["v"]).max())
        print(f"potential {pot} m {m} scheme {scheme}: {e:.2e}")
        assert e <= tol, (pot, e)


def test_f64_fig2_one_step_from_shared_states(gpu):
    sde, ctx, dev = gpu
    pt = dict(sde_inputs.jj_fig2(n_paths=1024)[0], n_steps=50)
    seed = sde_inputs.seed_of(11)
    ref = oracle.jj_integrate([pt], seed, n_record=50)
    init = oracle.jj_integrate([dict(pt, n_steps=0)], seed)
    xs = [init["phi"]] + list(ref["rec_phi"])
    vs = [init["v"]] + list(ref["rec_v"])
    worst = 0.0
    for k in range(50):
        w = np.floor(xs[k])
        st = (torch.from_numpy(xs[k] - w).to(dev), torch.from_numpy(w.astype(np.int32)).to(dev),
              torch.from_numpy(vs[k].copy()).to(dev), torch.zeros(1024, dtype=torch.float64, device=dev))
        st, _ = _run64(gpu, [dict(pt, n_steps=1)], seed, step0=k, state=st, sums=False)
        e = max(rel_err(_coord(st, 1.0), xs[k + 1]).max(), rel_err(st[2].cpu().numpy(), vs[k + 1]).max())
        worst = max(worst, e)
        assert e <= 1e-13, (k, e)
    print(f"FP64 worst one-step relative error: {worst:.2e}")


def test_f64_resume_bit_identical(gpu):
    """A run split at a step that is a multiple of 4 (one Philox block) and
    of M reproduces the single call bit for bit; a split elsewhere re-wraps
    the phase and folds the window sum at the boundary, so it agrees to
    rounding only."""
    pts = sde_inputs.jj_single(n_paths=300, n_steps=1000)
    a, psa = _run64(gpu, pts, 8)
    b, _ = _run64(gpu, [dict(pts[0], n_steps=400)], 8)
    b, psb = _run64(gpu, [dict(pts[0], n_steps=600)], 8, step0=400, state=b)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    assert torch.equal(psa, psb)
    c, _ = _run64(gpu, [dict(pts[0], n_steps=437)], 8)
    c, psc = _run64(gpu, [dict(pts[0], n_steps=563)], 8, step0=437, state=c)
    assert rel_err(_coord(c, 2 * np.pi), _coord(a, 2 * np.pi)).max() <= 1e-12
    assert rel_err(c[2].cpu().numpy(), a[2].cpu().numpy()).max() <= 1e-12
    torch.testing.assert_close(psc, psa, rtol=1e-12, atol=1e-12)


def test_f64_fig2_mean_velocity(gpu):
    pt = dict(sde_inputs.jj_fig2(n_paths=2048)[0], n_steps=20000, n_transient=10000)
    seed = sde_inputs.seed_of(13)
    st, ps = _run64(gpu, [pt], seed)
    ref = oracle.jj_integrate([pt], seed)
    g, r = st[3].cpu().numpy() / 10000, ref["acc"] / 10000
    d = g - r
    se = d.std(ddof=1) / np.sqrt(d.size)
    print(f"<v> FP64 gpu {g.mean():.5f} oracle {r.mean():.5f} diff {d.mean():.2e} SE {se:.2e}")
    assert abs(d.mean()) <= 3 * se + 1e-4
    np.testing.assert_allclose(ps.cpu().numpy()[0], [g.sum(), (g ** 2).sum()], rtol=1e-12)


def test_single_vs_double_precision_histograms(gpu):
    """Fig. 2 point, 2^15 paths, 200 periods: the coarse-grained position
    histograms of the FP32 and FP64 runs (same noise) agree within the
    statistical error, and so do the mean velocities."""
    sde, ctx, dev = gpu
    pt = dict(sde_inputs.jj_fig2(n_paths=1 << 15)[0], n_steps=20000)
    seed = sde_inputs.seed_of(15)
    n = pt["n_paths"]
    s32 = _state(n, dev, torch.float32)
    sde.sde_jj_integrate(ctx, [pt], sde.make_run(seed, sync=1), *s32)
    s64, _ = _run64(gpu, [pt], seed, sums=False)
    x0 = int(s64[1].median().item()) - 100
    h = []
    for st in (s32, s64):
        c = torch.zeros(202, dtype=torch.int64, device=dev)
        sde.sde_position_histogram(ctx, st[1], x0, 200, c)
        torch.cuda.synchronize()
        h.append(c.cpu().numpy())
    keep = (h[0] + h[1]) >= 10
    a, b = h[0][keep], h[1][keep]
    chi2 = float((((a - b) ** 2) / (a + b)).sum())
    p = stats.chi2.sf(chi2, keep.sum() - 1)
    v32, v64 = s32[3].cpu().numpy() / 20000, s64[3].cpu().numpy() / 20000
    se = np.hypot(v32.std(ddof=1), v64.std(ddof=1)) / np.sqrt(n)
    print(f"SP vs DP: chi2 {chi2:.1f} on {keep.sum() - 1} dof (p = {p:.3g}); <v> {v32.mean():.5f} vs "
          f"{v64.mean():.5f} (SE {se:.1e}); paths with the same final winding: "
          f"{np.mean(s32[1].cpu().numpy() == s64[1].cpu().numpy()):.3f}")
    assert p > 1e-4
    assert abs(v32.mean() - v64.mean()) <= 4 * se + 1e-4


def test_f64_invalid_arguments(gpu):
    sde, ctx, dev = gpu
    pt = sde_inputs.jj_point(n_paths=64, n_steps=10)
    st = _state(64, dev)
    # theta 4 bytes off its 8-byte alignment: rejected before any launch
    with pytest.raises(sde.SDEError) as e:
        sde.sde_jj_integrate_f64(ctx, [pt], sde.make_run(1, sync=1), st[0].data_ptr() + 4, st[1], st[2], st[3])
    assert e.value.status == sde.SDE_ERR_INVALID
