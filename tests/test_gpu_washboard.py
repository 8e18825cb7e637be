"""GPU parity of the paper's own form of Eq. 1 -- V(x) = sin(2 pi x), x in
potential periods (Sec. 3, Fig. 2) -- and of the coarse-grained position
histogram (one bin per period), through the C ABI.

Tolerances:
  * one step from a shared state (the oracle's FP64 state rounded to FP32),
    every step of the first 100: relative error |d| / max(|ref|, 1) <= 1e-5
    on x = theta + winding and on v.  Trajectories are compared step by step
    rather than over 100 steps because the barrier tops of this potential
    are unstable at a rate of about 2 pi per unit time (4 pi^2 / gamma when
    overdamped): over 100 steps of the Fig. 2 discretization a path near a
    barrier amplifies FP32 rounding ~10^3-fold, a property of the dynamics
    (a float32 replica of the kernel arithmetic on the CPU shows the same);
  * short trajectories where the amplification stays small (400 steps per
    period, 100 steps, inertial): <= 1e-5 per path;
  * ensemble mean velocity: paired |gpu - oracle| <= 3 SE + 1e-4;
  * histograms: bit-exact against numpy on the same windings (integer work);
    GPU against oracle ensembles: two-sample chi-square, p > 1e-4.
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


def _state(n, dev):
    return (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float64, device=dev))


def _x(st):
    return st[0].cpu().double().numpy() + st[1].cpu().double().numpy()


def _run(gpu, pts, seed, step0=0, scheme=0, state=None, sums=True):
    sde, ctx, dev = gpu
    n = sum(p["n_paths"] for p in pts)
    init = sde.SDE_INIT_FROM_STATE if state is not None else sde.SDE_INIT_PHILOX
    st = state if state is not None else _state(n, dev)
    ps = torch.zeros((len(pts), 2), dtype=torch.float64, device=dev) if sums else None
    sde.sde_jj_integrate(ctx, pts, sde.make_run(seed, step0=step0, scheme=scheme, init=init, sync=1), *st, ps)
    return st, ps


def _from_oracle(x, v, dev):
    """The oracle's FP64 state as the library's (theta, winding, v, acc)."""
    w = np.floor(x)
    th = (x - w).astype(np.float32)
    # rounding can push theta to 1.0f: carry it into the winding
    wrap = th >= 1.0
    th[wrap] = 0.0
    w[wrap] += 1
    return (torch.from_numpy(th).to(dev), torch.from_numpy(w.astype(np.int32)).to(dev),
            torch.from_numpy(v.astype(np.float32)).to(dev), torch.zeros(x.size, dtype=torch.float64, device=dev))


def _one_step_parity(gpu, pt, seed, scheme, n_check=100):
    sde, ctx, dev = gpu
    ref = oracle.jj_integrate([pt], seed, scheme=scheme, n_record=n_check)
    init = oracle.jj_integrate([dict(pt, n_steps=0)], seed)
    xs = [init["phi"]] + [ref["rec_phi"][k] for k in range(n_check)]
    vs = [init["v"]] + [ref["rec_v"][k] for k in range(n_check)]
    worst = 0.0
    for k in range(n_check):
        st = _from_oracle(xs[k], vs[k], dev)
        st, _ = _run(gpu, [dict(pt, n_steps=1)], seed, step0=k, scheme=scheme, state=st, sums=False)
        e = max(rel_err(_x(st), xs[k + 1]).max(), rel_err(st[2].cpu().double().numpy(), vs[k + 1]).max())
        worst = max(worst, e)
        assert e <= 1e-5, (k, e)
    print(f"worst one-step relative error: {worst:.2e}")


def test_sin2pi_fig2_one_step_from_shared_states(gpu):
    """The Fig. 2 point (dt = 0.01 of the drive period), 2048 paths."""
    pt = dict(sde_inputs.jj_fig2(n_paths=2048)[0], n_steps=100)
    _one_step_parity(gpu, pt, sde_inputs.seed_of(11), scheme=0)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("m", [1.0, 0.0])
def test_sin2pi_schemes_and_overdamped_one_step(gpu, scheme, m):
    pt = sde_inputs.jj_point(m=m, gamma=0.9 if m else 1.3, f=0.3 if m else 7.0, D=0.01, n_paths=1000,
                             steps_per_period=200, n_steps=60, potential=P2)
    _one_step_parity(gpu, pt, 5, scheme=scheme, n_check=60)


def test_sin2pi_short_trajectory_per_path(gpu):
    """400 steps per period, 100 steps in one call, 4096 paths."""
    pt = sde_inputs.jj_point(n_paths=4096, steps_per_period=400, n_steps=100, potential=P2)
    seed = sde_inputs.seed_of(12)
    st, _ = _run(gpu, [pt], seed, sums=False)
    ref = oracle.jj_integrate([pt], seed)
    e = max(rel_err(_x(st), ref["phi"]).max(), rel_err(st[2].cpu().double().numpy(), ref["v"]).max())
    print(f"100-step per-path relative error: {e:.2e}")
    assert e <= 1e-5


def _paired_ok(g, r, what):
    d = np.asarray(g, dtype=np.float64) - np.asarray(r, dtype=np.float64)
    se = d.std(ddof=1) / np.sqrt(d.size)
    print(f"{what}: gpu {np.mean(g):.5f} oracle {np.mean(r):.5f} diff {d.mean():.2e} SE {se:.2e}")
    assert abs(d.mean()) <= 3 * se + 1e-4, what


def test_sin2pi_fig2_mean_velocity(gpu):
    """Fig. 2 point, 2048 paths, 200 periods (100 transient): the paired time-
    and ensemble-averaged velocity, and the per-point sums."""
    pt = dict(sde_inputs.jj_fig2(n_paths=2048)[0], n_steps=20000, n_transient=10000)
    seed = sde_inputs.seed_of(13)
    st, ps = _run(gpu, [pt], seed)
    ref = oracle.jj_integrate([pt], seed)
    _paired_ok(st[3].cpu().numpy() / 10000, ref["acc"] / 10000, "<v>")
    vb = st[3].cpu().numpy() / 10000
    np.testing.assert_allclose(ps.cpu().numpy()[0], [vb.sum(), (vb ** 2).sum()], rtol=1e-12)


def _hist_np(w, x0, nb):
    w = np.asarray(w, dtype=np.int64)
    out = np.zeros(nb + 2, dtype=np.uint64)
    out[0] = np.count_nonzero(w < x0)
    out[nb + 1] = np.count_nonzero(w >= x0 + nb)
    inside = w[(w >= x0) & (w < x0 + nb)] - x0
    out[1:nb + 1] = np.bincount(inside, minlength=nb).astype(np.uint64)
    return out


@pytest.mark.parametrize("n,x0,nb", [(0, 0, 200), (1, -5, 1), (1000, -100, 200), (257 * 1031, -300, 200),
                                     (3_000_001, -2_000_000_000, 9000), (100_000, 7, 1 << 16)])
def test_histogram_bit_exact(gpu, n, x0, nb):
    """Random windings spanning both sides of the bin range, LDS bins and the
    global-atomics path (n_bins + 2 > 8192), ragged sizes, an empty input."""
    sde, ctx, dev = gpu
    rng = np.random.default_rng(n + nb)
    w = rng.integers(x0 - nb // 2 - 3, x0 + nb + nb // 2 + 3, n, dtype=np.int64)
    if n:
        w[0] = np.iinfo(np.int32).min
        w[-1] = np.iinfo(np.int32).max
    w = np.clip(w, np.iinfo(np.int32).min, np.iinfo(np.int32).max).astype(np.int32)
    wt = torch.from_numpy(w).to(dev)
    counts = torch.full((nb + 2,), 12345, dtype=torch.int64, device=dev)
    sde.sde_position_histogram(ctx, wt, x0, nb, counts)
    torch.cuda.synchronize()
    got = counts.cpu().numpy().view(np.uint64)
    assert np.array_equal(got, _hist_np(w, x0, nb))
    assert int(got.sum()) == n


def test_fig2_histogram_gpu_vs_oracle(gpu):
    """Fig. 2 point, 2^14 paths, 100 periods: the GPU ensemble's 200-bin
    histogram (bin = one period, centred on the ensemble) equals numpy's
    histogram of the same windings, and matches the oracle ensemble's."""
    sde, ctx, dev = gpu
    pt = dict(sde_inputs.jj_fig2(n_paths=1 << 14)[0], n_steps=10000)
    seed = sde_inputs.seed_of(14)
    st, _ = _run(gpu, [pt], seed, sums=False)
    ref = oracle.jj_integrate([pt], seed)
    w_gpu = st[1].cpu().numpy()
    x0 = int(np.floor(np.median(ref["phi"]))) - 100
    counts = torch.zeros(202, dtype=torch.int64, device=dev)
    sde.sde_position_histogram(ctx, st[1], x0, 200, counts)
    torch.cuda.synchronize()
    h_gpu = counts.cpu().numpy().view(np.uint64).astype(np.int64)
    assert np.array_equal(h_gpu, _hist_np(w_gpu, x0, 200).astype(np.int64))
    h_orc = _hist_np(np.floor(ref["phi"]).astype(np.int64), x0, 200).astype(np.int64)
    keep = (h_gpu + h_orc) >= 10
    a, b = h_gpu[keep], h_orc[keep]
    chi2 = float((((a - b) ** 2) / (a + b)).sum())
    p = stats.chi2.sf(chi2, keep.sum() - 1)
    print(f"histogram chi2 {chi2:.1f} on {keep.sum() - 1} dof, p = {p:.3g}; occupied bins {keep.sum()}")
    assert p > 1e-4


def test_mixed_kinds_in_one_call(gpu):
    """Points of both potentials, inertial and overdamped, in one call: each
    equals the same point integrated alone (same point index in the noise
    counters) bit for bit; the point sums group paths by the launch's
    paths-per-lane choice, so they agree to rounding."""
    sde, ctx, dev = gpu
    pts = [sde_inputs.jj_point(m=m, gamma=1.1, f=f, D=0.01, n_paths=np_, steps_per_period=200, n_steps=ns,
                               potential=pot)
           for m, f, np_, ns, pot in [(1.0, 0.2, 300, 500, 0), (0.0, 1.2, 70, 300, 0), (1.0, 0.1, 129, 400, 1),
                                      (0.0, 7.0, 64, 250, 1), (1.0, 0.3, 33, 600, 1)]]
    seed = 21
    st, ps = _run(gpu, pts, seed)
    assert sde.sde_get_stats(ctx)["work_items"] >= len(pts)
    off = 0
    for q, pt in enumerate(pts):
        n = pt["n_paths"]
        # alone, as point q of a batch whose earlier points have no paths in
        # it: the Philox counter uses the point index q
        solo = [dict(p, n_steps=0) for p in pts[:q]] + [pt]
        st1, ps1 = _run(gpu, solo, seed)
        o1 = sum(p["n_paths"] for p in pts[:q])
        for a, b in zip(st, st1):
            assert torch.equal(a[off:off + n], b[o1:o1 + n]), q
        torch.testing.assert_close(ps[q], ps1[q], rtol=1e-12, atol=1e-12)
        off += n


def test_potential_validation_leaves_outputs(gpu):
    sde, ctx, dev = gpu
    for bad in (dict(potential=2), dict(potential=-1), dict(reserved=1)):
        pt = dict(sde_inputs.jj_point(n_paths=64, n_steps=10), **bad)
        arr = sde.make_points([pt])
        if "reserved" in bad:
            arr[0].reserved = 1
        st = _state(64, dev)
        for x in st:
            x.zero_()
        with pytest.raises(sde.SDEError) as e:
            sde.sde_jj_integrate(ctx, arr, sde.make_run(1, sync=1), *st)
        assert e.value.status == sde.SDE_ERR_INVALID
        assert all(torch.count_nonzero(x) == 0 for x in st)


def test_fig2_full_size_one_step(gpu):
    """The Fig. 2 ensemble at its full size (2^19 paths, the benchmark's
    launch): one step from the oracle's state after 49 steps, every path,
    FP32 (1e-5) and FP64 (1e-13), against the oracle's step 50."""
    sde, ctx, dev = gpu
    pt = dict(sde_inputs.jj_fig2()[0], n_steps=49)
    seed = sde_inputs.seed_of(20)
    s49 = oracle.jj_integrate([pt], seed)
    s50 = oracle.jj_integrate([dict(pt, n_steps=1)], seed, step0=49, state=(s49["phi"], s49["v"], s49["acc"]))
    n = pt["n_paths"]
    st = _from_oracle(s49["phi"], s49["v"], dev)
    st, _ = _run(gpu, [dict(pt, n_steps=1)], seed, step0=49, state=st, sums=False)
    e32 = max(rel_err(_x(st), s50["phi"]).max(), rel_err(st[2].cpu().double().numpy(), s50["v"]).max())
    w = np.floor(s49["phi"])
    st64 = (torch.from_numpy(s49["phi"] - w).to(dev), torch.from_numpy(w.astype(np.int32)).to(dev),
            torch.from_numpy(s49["v"].copy()).to(dev), torch.zeros(n, dtype=torch.float64, device=dev))
    sde.sde_jj_integrate_f64(ctx, [dict(pt, n_steps=1)], sde.make_run(seed, step0=49, init=sde.SDE_INIT_FROM_STATE,
                                                                        sync=1), *st64)
    x64 = st64[0].cpu().numpy() + st64[1].cpu().numpy().astype(np.float64)
    e64 = max(rel_err(x64, s50["phi"]).max(), rel_err(st64[2].cpu().numpy(), s50["v"]).max())
    print(f"Fig. 2 at 2^19 paths, one step: FP32 {e32:.2e}, FP64 {e64:.2e}")
    assert e32 <= 1e-5
    assert e64 <= 1e-13
