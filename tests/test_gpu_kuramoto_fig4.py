"""The mean field streamed through HBM (realizations too large for registers,
Fig. 4: 2^24 identical oscillators) and the phase density P(x; t).

Checks:
  * the streamed variant (forced on at sizes the oracle finishes in
    seconds) against the FP64 oracle, first 100 steps under shared noise,
    Heun and Euler-Maruyama, per oscillator: circular |d phi| <= 1e-5
    max(|phi|, 1) (as the register-resident kernel); order parameter samples
    to 1e-6; several cooperative launches (R above the co-resident limit);
  * the streamed and register-resident variants agree to twice that bound
    on the uniform workload (N = 65536, 16 realizations, 100 steps);
  * Fig. 4 at its size (N = 2^24, omega = 0, K = 4, D = 1): one step from a
    shared state against the oracle for every oscillator (the oracle takes
    one step of 2^24 oscillators in FP64 in seconds); the late order
    parameter against the self-consistency r = I1(K r/D)/I0(K r/D) = 0.83146
    (K/D = 4); the late phase density against the stationary density
    exp(kappa cos 2 pi (theta - psi)) / I0(kappa), kappa = K r / D, within 2 %
    of its peak per bin (the counting noise is ~0.1 % there);
  * phase histograms bit-exact against numpy's floor(float64(theta) n_bins)
    with theta = 1 in the last bin and anything outside [0, 1] or NaN in the
    extra bin.
"""
import numpy as np
import pytest
import torch
from scipy import special

import oracle
import sde_inputs

pytestmark = pytest.mark.gpu

R_STAR = 0.8314620247541972  # r = I1(4 r) / I0(4 r)


def _circ_err(theta_gpu, phi_ref):
    d = 2 * np.pi * theta_gpu.astype(np.float64) - phi_ref
    d = np.mod(d + np.pi, 2 * np.pi) - np.pi
    return np.abs(d) / np.maximum(np.abs(phi_ref), 1.0)


def _run(gpu, N, R, K, D, dt, n_steps, scheme=0, seed=1, omega=None, phi=None, step0=0, M=100, streamed=True,
         samples=True, opt=0, paired=0):
    """paired: 0 as tuned, 1 one realization per workgroup, 2 two."""
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF, 1 if streamed else 2)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_OPT, opt)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_PAIRED, paired)
    om = omega if isinstance(omega, torch.Tensor) else torch.from_numpy(np.asarray(omega, dtype=np.float32)).to(dev)
    if phi is None:
        ph = torch.empty((R, N), dtype=torch.float32, device=dev)
        init = sde.SDE_INIT_PHILOX
    else:
        ph = phi
        init = sde.SDE_INIT_FROM_STATE
    rs = torch.zeros((R, n_steps // M + 1), dtype=torch.float64, device=dev) if samples else None
    desc = sde.sde_kuramoto_desc(N, R, K, D, dt, n_steps, sde.SDE_MEANFIELD, 0)
    run = sde.make_run(seed, step0=step0, scheme=scheme, init=init, sample_every=M, sync=1)
    sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, None, rs)
    st = sde.sde_get_stats(ctx)
    assert st["mf_streamed"] == (1 if streamed else 0)
    if opt:
        assert st["kura_mf_opt"] == opt
    if paired:
        assert st["kura_mf_paired"] == paired - 1
    return ph, rs


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("N,R", [(65536, 16), (3000, 3), (1000, 300)])
def test_streamed_first_100_steps(gpu, scheme, N, R):
    """Ragged slices (N not a multiple of the slice), several workgroups per
    realization, and R = 300 > the co-resident workgroups (two launches)."""
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, scheme, cfg["seed"], cfg["omega"])
    ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD,
                                          scheme, cfg["seed"], cfg["omega"].astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"streamed mean field N {N} R {R} scheme {scheme}: max phase error {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


@pytest.mark.parametrize("streamed,N", [(True, 1 << 17), (False, 1 << 18)])
def test_tree_exchange_vs_oracle(gpu, streamed, N):
    """2 realizations of N = 2^17 streamed (128 workgroups per realization)
    or N = 2^18 in registers (64 workgroups of 512 lanes x 8 oscillators),
    so the sums go through the two-level exchange (group leaders, then the
    8 group sums); first 100 steps against the oracle."""
    R = 2
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    for scheme in (0, 1):
        ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, scheme, cfg["seed"], cfg["omega"],
                      streamed=streamed, opt=0 if streamed else 8, paired=0 if streamed else 1)
        ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD,
                                              scheme, cfg["seed"], cfg["omega"].astype(np.float64))
        err = _circ_err(ph.cpu().numpy(), ref)
        print(f"tree exchange, streamed {streamed}, scheme {scheme}: max phase error {err.max():.2e}")
        assert err.max() <= 1e-5
        np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


@pytest.mark.parametrize("N,opt", [(12289, 2), (30001, 4), (65535, 8), (100003, 8), (12289, 1), (700, 2),
                                   (4000, 8), (512, 1)])
def test_register_resident_lane_counts(gpu, N, opt):
    """The register-resident kernel at each count of oscillators per lane,
    forced, the last workgroup ragged: N = 100003 needs 25 workgroups of 8
    per lane, rounded up to 32 for the two-level exchange, the last 7 empty;
    12289 at 1 per lane also takes the two-level exchange (25 -> 32);
    700, 4000 and 512 fit one workgroup (no exchange).  Heun and
    Euler-Maruyama, 3 realizations."""
    R = 3
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    for scheme in (0, 1):
        ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, scheme, cfg["seed"], cfg["omega"],
                      streamed=False, opt=opt, paired=1)
        ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD,
                                              scheme, cfg["seed"], cfg["omega"].astype(np.float64))
        err = _circ_err(ph.cpu().numpy(), ref)
        print(f"registers, N {N}, {opt} per lane, scheme {scheme}: max phase error {err.max():.2e}")
        assert err.max() <= 1e-5
        np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_meanfield_tuner(gpu):
    """With the lane count left to the tuner, the first call of a shape class
    times the fitting counts and caches the choice; the next call of the
    class reuses it without tuning and equals, bit for bit, a run forced to
    that count.  A count at which N does not fit is refused."""
    sde, ctx, dev = gpu
    N, R = 8197, 5
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    args = (N, R, cfg["K"], cfg["D"], cfg["dt"], 50, 0, cfg["seed"], cfg["omega"])
    _run(gpu, *args, streamed=False)
    st1 = sde.sde_get_stats(ctx)
    assert st1["tuned"] == 1 and st1["kura_mf_opt"] in (1, 2, 4, 8)
    a, ra = _run(gpu, *args, streamed=False)
    st2 = sde.sde_get_stats(ctx)
    assert st2["tuned"] == 0 and st2["kura_mf_opt"] == st1["kura_mf_opt"]
    assert st2["kura_mf_paired"] == st1["kura_mf_paired"]
    b, rb = _run(gpu, *args, streamed=False, opt=st1["kura_mf_opt"], paired=1 + st1["kura_mf_paired"])
    assert torch.equal(a, b) and torch.equal(ra, rb)
    print(f"mean-field tuner: {st1['kura_mf_opt']} per lane, paired {st1['kura_mf_paired']} for N {N}, R {R} "
          f"({st1['tune_ms']:.2f} ms)")
    for bad in (3, 16, -1):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_OPT, bad)
    for bad in (3, -1):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_PAIRED, bad)
    # 2^18 oscillators at 1 per lane would need 512 workgroups per realization
    Nb = 1 << 18
    ph = torch.zeros((1, Nb), dtype=torch.float32, device=dev)
    om = torch.zeros(Nb, dtype=torch.float32, device=dev)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF, 2)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_OPT, 1)
    desc = sde.sde_kuramoto_desc(Nb, 1, 1.0, 0.1, 0.01, 10, sde.SDE_MEANFIELD, 0)
    with pytest.raises(sde.SDEError) as e:
        sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(1, sync=1), ph, om, None, None)
    assert e.value.status == sde.SDE_ERR_UNSUPPORTED
    assert torch.count_nonzero(ph) == 0


@pytest.mark.parametrize("N,opt,R", [(65536, 4, 4), (12289, 2, 2), (30001, 4, 6), (700, 2, 2), (20000, 2, 4)])
def test_two_realizations_per_workgroup(gpu, N, opt, R):
    """The kernel that holds two realizations per workgroup (and a ninth
    wave for the exchanges), forced: N = 65536 at 4 per lane is 32
    workgroups per realization (two polled words per lane), 20000 at 2 per
    lane 20, 12289 and 30001 13 and 15 (ragged), 700 a single workgroup (no
    exchange); R = 6 is three pairs.  Heun and Euler-Maruyama against the
    oracle over 100 steps, as the one-realization kernel."""
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    for scheme in (0, 1):
        ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, scheme, cfg["seed"], cfg["omega"],
                      streamed=False, opt=opt, paired=2)
        ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD,
                                              scheme, cfg["seed"], cfg["omega"].astype(np.float64))
        err = _circ_err(ph.cpu().numpy(), ref)
        print(f"two per workgroup, N {N}, {opt} per lane, R {R}, scheme {scheme}: max phase error {err.max():.2e}")
        assert err.max() <= 1e-5
        np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_two_realizations_resume_and_limits(gpu):
    """Two realizations per workgroup: a run split in two calls equals the
    whole run bit for bit, a repeated run is identical, and an odd R or a
    slice of more than 32 workgroups is refused when forced."""
    sde, ctx, dev = gpu
    N, R = 3000, 4
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    base = (N, R, cfg["K"], cfg["D"], cfg["dt"])
    full, rf = _run(gpu, *base, 50, 0, 5, cfg["omega"], streamed=False, paired=2, samples=False)
    again, _ = _run(gpu, *base, 50, 0, 5, cfg["omega"], streamed=False, paired=2, samples=False)
    a, _ = _run(gpu, *base, 21, 0, 5, cfg["omega"], streamed=False, paired=2, samples=False)
    b, _ = _run(gpu, *base, 29, 0, 5, cfg["omega"], phi=a, step0=21, streamed=False, paired=2, samples=False)
    assert torch.equal(full, again) and torch.equal(full, b)
    om = torch.zeros(N, dtype=torch.float32, device=dev)
    for n_, r_, opt in [(N, 3, 0), (1 << 17, 2, 2)]:
        ph = torch.zeros((r_, n_), dtype=torch.float32, device=dev)
        om = torch.zeros(n_, dtype=torch.float32, device=dev)
        sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF, 2)
        sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_OPT, opt)
        sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF_PAIRED, 2)
        desc = sde.sde_kuramoto_desc(n_, r_, 1.0, 0.1, 0.01, 10, sde.SDE_MEANFIELD, 0)
        with pytest.raises(sde.SDEError) as e:
            sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(1, sync=1), ph, om, None, None)
        assert e.value.status == sde.SDE_ERR_UNSUPPORTED
        assert torch.count_nonzero(ph) == 0


def test_streamed_matches_register_resident(gpu):
    """Both variants are within 1e-5 of the oracle after 100 steps, so within
    2e-5 of each other (they round differently: the carry form, the slice
    sizes of the sums)."""
    cfg = sde_inputs.kuramoto_uniform()
    N, R = cfg["N"], cfg["R"]
    a, ra = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 0, cfg["seed"], cfg["omega"], streamed=True)
    b, rb = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 0, cfg["seed"], cfg["omega"], streamed=False)
    err = _circ_err(a.cpu().numpy(), 2 * np.pi * b.cpu().numpy().astype(np.float64))
    print(f"streamed vs registers, 100 steps: max phase difference {err.max():.2e}")
    assert err.max() <= 2e-5
    np.testing.assert_allclose(ra.cpu().numpy(), rb.cpu().numpy(), rtol=0, atol=2e-6)


def test_streamed_resume_bit_identical(gpu):
    cfg = sde_inputs.kuramoto_uniform(N=5000, R=4)
    args = (5000, 4, cfg["K"], cfg["D"], cfg["dt"])
    full, _ = _run(gpu, *args, 50, 0, 8, cfg["omega"], samples=False)
    a, _ = _run(gpu, *args, 21, 0, 8, cfg["omega"], samples=False)
    b, _ = _run(gpu, *args, 29, 0, 8, cfg["omega"], phi=a, step0=21, samples=False)
    assert torch.equal(full, b)


def _stationary_density(n_bins, kappa, psi):
    """Bin averages of exp(kappa cos 2 pi (theta - psi)) / I0(kappa) on [0, 1)."""
    edges = np.arange(n_bins + 1) / n_bins
    x = edges[:-1, None] + (np.arange(64)[None, :] + 0.5) / (64 * n_bins)
    f = np.exp(kappa * (np.cos(2 * np.pi * (x - psi)) - 1.0)) / special.i0e(kappa)
    return f.mean(axis=1)


def test_fig4_two_to_the_24(gpu):
    sde, ctx, dev = gpu
    cfg = sde_inputs.kuramoto_fig4(n_steps=3000)
    N, K, D, dt = cfg["N"], cfg["K"], cfg["D"], cfg["dt"]
    om = torch.zeros(N, dtype=torch.float32, device=dev)
    # one step from the Philox initial state and from the late state, every oscillator
    ph0, _ = _run(gpu, N, 1, K, D, dt, 0, 0, cfg["seed"], om, samples=False)
    ph, rs = _run(gpu, N, 1, K, D, dt, cfg["n_steps"], 0, cfg["seed"], om)
    zeros = np.zeros(N)
    for name, state, k in [("initial", ph0, 0), ("late", ph, cfg["n_steps"])]:
        one, _ = _run(gpu, N, 1, K, D, dt, 1, 0, cfg["seed"], om, phi=state.clone(), step0=k, samples=False)
        ref, _ = oracle.kuramoto_integrate(N, 1, K, D, dt, 1, 0, oracle.MEANFIELD, 0, cfg["seed"], zeros,
                                           phi0=2 * np.pi * state.cpu().numpy().astype(np.float64), step0=k)
        err = _circ_err(one.cpu().numpy(), ref)
        print(f"Fig. 4, one step from the {name} state: max phase error {err.max():.2e}")
        assert err.max() <= 1e-5
    r = rs.cpu().numpy()[0]
    r_late = r[-10:].mean()
    print(f"Fig. 4: r(0) = {r[0]:.5f}, r(t) every 100 steps ... late mean {r_late:.5f} (self-consistency {R_STAR:.5f})")
    assert r[0] < 0.01
    assert abs(r_late - R_STAR) <= 3e-3
    n_bins = 100
    counts = torch.zeros((1, n_bins + 1), dtype=torch.int64, device=dev)
    sde.sde_phase_histograms(ctx, ph, n_bins, counts)
    torch.cuda.synchronize()
    h = counts.cpu().numpy()[0]
    assert h[n_bins] == 0 and h.sum() == N
    th = ph.cpu().numpy().astype(np.float64)[0]
    psi = np.arctan2(np.sin(2 * np.pi * th).sum(), np.cos(2 * np.pi * th).sum()) / (2 * np.pi)
    dens = h[:n_bins] * n_bins / N
    ref = _stationary_density(n_bins, K * R_STAR / D, psi)
    dev_max = np.abs(dens - ref).max() / ref.max()
    print(f"Fig. 4 late density: max deviation {dev_max:.3%} of the peak {ref.max():.3f}")
    assert dev_max <= 0.02


def _phase_hist_np(t, nb):
    t = np.asarray(t, dtype=np.float32)
    out = np.zeros(nb + 1, dtype=np.int64)
    ok = (t >= 0) & (t <= 1)
    b = np.minimum(np.floor(t[ok].astype(np.float64) * nb).astype(np.int64), nb - 1)
    out[:nb] = np.bincount(b, minlength=nb)
    out[nb] = np.count_nonzero(~ok)
    return out


@pytest.mark.parametrize("rows,n,pitch,nb", [(1, 1000, 1000, 100), (5, 777, 800, 7), (3, 4000, 4000, 9000),
                                             (70000, 3, 3, 4), (2, 0, 4, 3)])
def test_phase_histograms_bit_exact(gpu, rows, n, pitch, nb):
    sde, ctx, dev = gpu
    rng = np.random.default_rng(rows * 7 + n + nb)
    t = rng.uniform(-0.1, 1.1, (rows, pitch)).astype(np.float32)
    specials = np.array([0.0, 1.0, np.nextafter(np.float32(1), np.float32(0)), -0.0, np.nan, np.inf, -1e-30,
                         1.0 / nb, 0.5], dtype=np.float32)
    if n >= len(specials):
        t[0, :len(specials)] = specials
    tt = torch.from_numpy(t).to(dev)
    counts = torch.full((rows, nb + 1), 5, dtype=torch.int64, device=dev)
    sde.sde_phase_histograms(ctx, tt, nb, counts, n=n)
    torch.cuda.synchronize()
    got = counts.cpu().numpy()
    for r in range(rows) if rows < 100 else list(range(50)) + list(range(rows - 50, rows)):
        assert np.array_equal(got[r], _phase_hist_np(t[r, :n], nb)), r
    assert (got.sum(axis=1) == n).all()
    with pytest.raises(sde.SDEError):
        sde.sde_phase_histograms(ctx, tt, 0, counts, n=n)


def test_mf_option_validation(gpu):
    sde, ctx, dev = gpu
    for bad in (-1, 3):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF, bad)
    # forcing the register-resident kernel past its size is reported, not run
    N = 1 << 21
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_MF, 2)
    ph = torch.zeros((1, N), dtype=torch.float32, device=dev)
    om = torch.zeros(N, dtype=torch.float32, device=dev)
    desc = sde.sde_kuramoto_desc(N, 1, 1.0, 0.1, 0.01, 10, sde.SDE_MEANFIELD, 0)
    with pytest.raises(sde.SDEError) as e:
        sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(1, sync=1), ph, om, None, None)
    assert e.value.status == sde.SDE_ERR_UNSUPPORTED
    assert torch.count_nonzero(ph) == 0
