"""GPU parity of the Josephson-junction path (Eq. 1 through Alg. 1/2)
against the FP64 oracle, through the C ABI.

Tolerances:
  * Philox words: bit-exact (integer work).
  * per-path state over the first 100 steps under shared noise: relative
    error |d| / max(|ref|, 1) <= 1e-5 on phi = 2 pi (theta + winding) and v;
  * ensemble observables: |gpu - oracle| <= 3 SE + 1e-4 (SE of the oracle's
    ensemble mean).
"""
import numpy as np
import pytest
import torch

import oracle
import sde_inputs
from conftest import rel_err

pytestmark = pytest.mark.gpu


def _state(n, dev):
    return (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float64, device=dev))


def _phi(theta, wind):
    return 2 * np.pi * (theta.cpu().double().numpy() + wind.cpu().double().numpy())


def _run(gpu, pts, seed, step0=0, scheme=0, state=None, M=0, sums=True):
    sde, ctx, dev = gpu
    n = sum(p["n_paths"] for p in pts)
    if state is None:
        state = _state(n, dev)
        init = sde.SDE_INIT_PHILOX
    else:
        init = sde.SDE_INIT_FROM_STATE
    ps = torch.zeros((len(pts), 2), dtype=torch.float64, device=dev) if sums else None
    run = sde.make_run(seed, step0=step0, scheme=scheme, init=init, sample_every=M, sync=1)
    sde.sde_jj_integrate(ctx, pts, run, *state, ps)
    return state, ps


@pytest.mark.parametrize("seed,tag,a,b,c0", [(0, 0, 0, 0, 0), (9033852, 0, 17, 3, 1000),
                                             (2**64 - 1, 1, 4095, 16383, 2**32 - 100)])
def test_philox_bit_exact(gpu, seed, tag, a, b, c0):
    sde, ctx, dev = gpu
    n = 1 << 16
    out = torch.empty((n, 4), dtype=torch.int32, device=dev)
    sde.sde_debug_philox(ctx, seed, tag, a, b, c0, n, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    ref = _stream_wrapped(seed, tag, a, b, c0, n)
    assert np.array_equal(got, ref)


def _stream_wrapped(seed, tag, a, b, c0, n):
    """Oracle blocks at counter word 0 = (c0 + k) mod 2^32."""
    first = min(n, 2**32 - c0)
    parts = [oracle.philox_stream(seed, tag, a, b, c0, first)]
    if first < n:
        parts.append(oracle.philox_stream(seed, tag, a, b, 0, n - first))
    return np.concatenate(parts)


def test_gaussians_match_oracle(gpu):
    """FP32 Box-Muller on the hardware log2/sqrt/sin/cos against FP64."""
    sde, ctx, dev = gpu
    n = 1 << 20
    out = torch.empty(n, dtype=torch.float32, device=dev)
    sde.sde_debug_gauss(ctx, 123, 0, 5, 7, 3, n, out)
    torch.cuda.synchronize()
    got = out.cpu().double().numpy()
    ref = oracle.gauss_array(123, 0, 5, 7, 3, n)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    print(f"gaussian max err {err.max():.3e}, 99.99% {np.quantile(err, 0.9999):.3e}")
    # 2e-6 max(1, |g|): the uniforms are exact in FP32; log2, sqrt, sin and
    # cos each round to about 1 ulp (2^-24 relative), the radius and the
    # products add a few more
    assert err.max() <= 2e-6


def test_jj_single_point_first_100_steps_per_path(gpu):
    """Per-path state after every step 1..100 (shared noise), 4096 paths."""
    pts = sde_inputs.jj_single(n_paths=4096, n_steps=100)
    seed = sde_inputs.seed_of(1)
    ref = oracle.jj_integrate(pts, seed, n_record=100)
    state = None
    worst = 0.0
    for k in range(100):
        one = [dict(pts[0], n_steps=1)]
        state, _ = _run(gpu, one, seed, step0=k, state=state, sums=False)
        phi = _phi(state[0], state[1])
        v = state[2].cpu().double().numpy()
        e = max(rel_err(phi, ref["rec_phi"][k]).max(), rel_err(v, ref["rec_v"][k]).max())
        worst = max(worst, e)
        assert e <= 1e-5, (k, e)
    print(f"worst per-path relative error over 100 steps: {worst:.2e}")
    # the same 100 steps in one call
    st2, _ = _run(gpu, pts, seed, sums=False)
    assert rel_err(_phi(st2[0], st2[1]), ref["phi"]).max() <= 1e-5
    assert rel_err(st2[2].cpu().double().numpy(), ref["v"]).max() <= 1e-5


def _paired_ok(g, r, what):
    """Ensemble means of paired per-path values agree within 3 SE of the
    mean difference + 1e-4 (both sides draw the same noise per path)."""
    d = np.asarray(g, dtype=np.float64) - np.asarray(r, dtype=np.float64)
    se = d.std(ddof=1) / np.sqrt(d.size) if d.size > 1 else 0.0
    print(f"{what}: gpu {np.mean(g):.6f} oracle {np.mean(r):.6f} diff {d.mean():.2e} SE {se:.2e}")
    assert abs(d.mean()) <= 3 * se + 1e-4, what


def test_jj_single_point_ensemble(gpu):
    """The full single-point workload: 4096 paths x 10^4 steps; <v> (time and
    ensemble average), <v(t_end)>, and the library's own reduction."""
    sde, ctx, dev = gpu
    pts = sde_inputs.jj_single()
    seed = sde_inputs.seed_of(1)
    state, ps = _run(gpu, pts, seed)
    ref = oracle.jj_integrate(pts, seed)
    P, W = pts[0]["n_paths"], pts[0]["n_steps"]
    _paired_ok(state[3].cpu().numpy() / W, ref["acc"] / W, "<v> time average")
    _paired_ok(state[2].cpu().double().numpy(), ref["v"], "<v(t_end)>")
    # the point sums are the per-path sums reduced on the device
    vb = state[3].cpu().numpy() / W
    np.testing.assert_allclose(ps.cpu().numpy()[0], [vb.sum(), (vb ** 2).sum()], rtol=1e-12)
    obs = sde.sde_observables(ctx, sde.SDE_OBS_MEAN_F32, state[2], [P])
    vg = state[2].cpu().double().numpy()
    np.testing.assert_allclose(obs[0], [vg.mean(), vg.std(ddof=1) / np.sqrt(P)], rtol=1e-10)


def test_jj_scan_slice(gpu):
    """Points of the (f, D) scan at its corners and middle, shortened to
    2*10^4 steps (10^4 transient) and 256 paths."""
    qs = [0, 127, 128 * 64 + 64, 128 * 127, 128 * 127 + 127, 128 * 30 + 100]
    pts = sde_inputs.jj_scan(n_paths=256, n_steps=20000, n_transient=10000, indices=qs)
    seed = sde_inputs.seed_of(2)
    st, ps = _run(gpu, pts, seed)
    ref = oracle.jj_integrate(pts, seed)
    acc = st[3].cpu().numpy()
    for q in range(len(qs)):
        sl = slice(256 * q, 256 * (q + 1))
        _paired_ok(acc[sl] / 10000, ref["acc"][sl] / 10000, f"point {qs[q]}")


def test_jj_scan_full_size_sampled(gpu):
    """The full (f, D) scan -- 16384 points x 1024 paths x 2*10^5 steps in
    one call, as the benchmark launches it -- checked on sampled points: the
    oracle integrates the first 48 paths of 6 points under their batch
    indices, and their time-averaged velocities are compared pairwise."""
    sde, ctx, dev = gpu
    pts = sde_inputs.jj_scan()
    seed = sde_inputs.seed_of(2)
    n = 16384 * 1024
    acc = torch.empty(n, dtype=torch.float64, device=dev)
    ps = torch.empty((16384, 2), dtype=torch.float64, device=dev)
    sde.sde_jj_integrate(ctx, pts, sde.make_run(seed, sync=1), None, None, None, acc, ps)
    sums = ps.cpu().numpy()
    assert np.all(np.isfinite(sums))
    vmean = sums[:, 0] / 1024
    assert np.all(np.abs(vmean) < 10.0)
    qs = [0, 4242, 8191, 9000, 12345, 16383]
    sub = [dict(pts[q], n_paths=48) for q in qs]
    ref = oracle.jj_integrate(sub, seed, point_ids=qs)
    a = acc.cpu().numpy()
    for i, q in enumerate(qs):
        g = a[1024 * q:1024 * q + 48] / 100000
        _paired_ok(g, ref["acc"][48 * i:48 * (i + 1)] / 100000, f"scan point {q}")
    # point sums agree with the per-path accumulators
    vb = a.reshape(16384, 1024) / 100000
    np.testing.assert_allclose(sums[:, 0], vb.sum(axis=1), rtol=1e-12, atol=1e-12)


def test_jj_resume_bit_identical(gpu):
    pts = sde_inputs.jj_scan(n_paths=300, n_steps=1000, n_transient=250, indices=[5, 9000])
    seed = 77
    full, ps_full = _run(gpu, pts, seed, M=100)
    a, _ = _run(gpu, [dict(p, n_steps=400) for p in pts], seed, M=100)
    b, ps_b = _run(gpu, [dict(p, n_steps=600) for p in pts], seed, step0=400, state=a, M=100)
    for x, y in zip(full, b):
        assert torch.equal(x, y)
    assert torch.equal(ps_full, ps_b)


def test_jj_deterministic(gpu):
    pts = sde_inputs.jj_scan(n_paths=1000, n_steps=500, n_transient=100, indices=range(0, 16384, 997))
    s1, p1 = _run(gpu, pts, 3)
    s2, p2 = _run(gpu, pts, 3)
    for x, y in zip(s1, s2):
        assert torch.equal(x, y)
    assert torch.equal(p1, p2)


def test_jj_ragged_uneven_unaligned(gpu):
    """Path counts that leave partial chunks, step counts that leave partial
    Philox blocks, an unaligned first step, zero-step points."""
    counts = [1, 63, 64, 65, 129, 300, 7]
    steps = [5, 0, 1, 203, 3, 97, 64]
    pts = [sde_inputs.jj_point(f=0.05 * i, D=1e-3 * (i + 1), n_paths=c, steps_per_period=50 + i,
                               n_steps=s, n_transient=10)
           for i, (c, s) in enumerate(zip(counts, steps))]
    seed = 11
    # start from the INIT state, advance 3 steps, then the uneven call from step 3
    st0, _ = _run(gpu, [dict(p, n_steps=3) for p in pts], seed, sums=False)
    ref0 = oracle.jj_integrate([dict(p, n_steps=3) for p in pts], seed)
    st, ps = _run(gpu, pts, seed, step0=3, state=st0)
    ref = oracle.jj_integrate(pts, seed, step0=3, state=(ref0["phi"], ref0["v"], ref0["acc"]))
    assert rel_err(_phi(st[0], st[1]), ref["phi"]).max() <= 1e-5
    assert rel_err(st[2].cpu().double().numpy(), ref["v"]).max() <= 1e-5
    np.testing.assert_allclose(st[3].cpu().numpy(), ref["acc"], rtol=1e-5, atol=1e-4)
    np.testing.assert_allclose(ps.cpu().numpy(), ref["point_sums"], rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("m", [1.0, 0.0])
def test_jj_schemes_and_overdamped(gpu, scheme, m):
    pts = [sde_inputs.jj_point(m=m, gamma=0.9 if m else 1.3, f=0.3 if m else 1.2, D=0.01,
                               n_paths=1000, n_steps=100)]
    seed = 5
    st, _ = _run(gpu, pts, seed, scheme=scheme, sums=False)
    ref = oracle.jj_integrate(pts, seed, scheme=scheme)
    assert rel_err(_phi(st[0], st[1]), ref["phi"]).max() <= 1e-5
    assert rel_err(st[2].cpu().double().numpy(), ref["v"]).max() <= 1e-5


def test_jj_invalid_arguments_leave_outputs(gpu):
    sde, ctx, dev = gpu
    good = sde_inputs.jj_point(n_paths=64, n_steps=10)
    st = _state(64, dev)
    for x in st:
        x.fill_(7)
    before = [x.clone() for x in st]
    bad_points = [dict(good, n_paths=0), dict(good, steps_per_period=0), dict(good, omega=0.0),
                  dict(good, gamma=-1.0), dict(good, D=-1e-3), dict(good, m=-1.0),
                  dict(good, a=float("nan")), dict(good, m=0.0, gamma=0.0)]
    for p in bad_points:
        with pytest.raises(sde.SDEError) as e:
            sde.sde_jj_integrate(ctx, [p], sde.make_run(1, sync=1), *st)
        assert e.value.status == sde.SDE_ERR_INVALID
    with pytest.raises(sde.SDEError):
        sde.sde_jj_integrate(ctx, [good], sde.make_run(1, scheme=5, sync=1), *st)
    with pytest.raises(sde.SDEError):
        sde.sde_jj_integrate(ctx, [good], sde.make_run(1, init=sde.SDE_INIT_FROM_STATE, sync=1),
                             st[0], None, st[2], st[3])
    with pytest.raises(sde.SDEError):
        sde.sde_jj_integrate(ctx, [good], sde.make_run(1, sync=1), st[0].data_ptr() + 2)
    torch.cuda.synchronize()
    for x, y in zip(st, before):
        assert torch.equal(x, y)


def test_jj_numeric_error_reported(gpu):
    sde, ctx, dev = gpu
    # one step per drive period of a slow drive: dt * gamma ~ 5e3, so the
    # explicit step amplifies v by ~1e7 per step and overflows to Inf/NaN
    p = sde_inputs.jj_point(omega=1e-3, steps_per_period=1, n_paths=64, n_steps=50)
    with pytest.raises(sde.SDEError) as e:
        _run(gpu, [p], 1)
    assert e.value.status == sde.SDE_ERR_NUMERIC
    # the flag is cleared: a good run afterwards succeeds
    _run(gpu, [sde_inputs.jj_point(n_paths=64, n_steps=50)], 1)


def test_observables_match_numpy(gpu):
    sde, ctx, dev = gpu
    rng = np.random.default_rng(0)
    counts = [1, 2, 255, 256, 257, 5000]
    x = rng.standard_normal(sum(counts)).astype(np.float32) * 3 + 1
    xt = torch.from_numpy(x).to(dev)
    out = sde.sde_observables(ctx, sde.SDE_OBS_MEAN_F32, xt, counts)
    sq = sde.sde_observables(ctx, sde.SDE_OBS_MEANSQ_F32, xt, counts)
    order = sde.sde_observables(ctx, sde.SDE_OBS_ORDER, xt, counts)
    xd = torch.from_numpy(x.astype(np.float64)).to(dev)
    out64 = sde.sde_observables(ctx, sde.SDE_OBS_MEAN_F64, xd, counts)
    o = 0
    for g, c in enumerate(counts):
        seg = x[o:o + c].astype(np.float64)
        o += c
        se = seg.std(ddof=1) / np.sqrt(c) if c > 1 else 0.0
        np.testing.assert_allclose(out[g], [seg.mean(), se], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(out64[g], [seg.mean(), se], rtol=1e-12, atol=1e-14)
        s2 = seg ** 2
        np.testing.assert_allclose(sq[g, 0], s2.mean(), rtol=1e-12)
        z = np.exp(2j * np.pi * seg).mean()
        np.testing.assert_allclose(order[g, 0], abs(z), rtol=1e-10, atol=1e-13)
