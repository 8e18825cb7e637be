"""GPU parity of the Kuramoto path (Eq. 2, Eq. 3, Alg. 3) against the FP64
oracle, through the C ABI.

Phases are compared on the circle: the GPU keeps theta = phi / 2 pi wrapped
to [0, 1), the oracle an unwrapped phi; the error is the circular distance
in radians.  Tolerances:
  * mean-field, tiled, dense FP32 and dense FP16x3, first 100 steps under
    shared noise: |d phi| <= 1e-5 max(|phi_ref|, 1) per oscillator;
  * dense BF16x3: the split product keeps ~16 mantissa bits per term, so
    the per-step drift error is bounded by 1.5 K 2^-15 ~ 2e-4 (worst case,
    all terms of one sign); over 100 steps of dt = 0.005 that is 1e-4 rad,
    the stated bound for that variant;
  * order parameter samples: paired differences within 3 SE + 1e-4.
"""
import numpy as np
import pytest
import torch

import oracle
import sde_inputs

pytestmark = pytest.mark.gpu


def _circ_err(theta_gpu, phi_ref):
    d = 2 * np.pi * theta_gpu.astype(np.float64) - phi_ref
    d = np.mod(d + np.pi, 2 * np.pi) - np.pi
    return np.abs(d) / np.maximum(np.abs(phi_ref), 1.0)


def _run(gpu, N, R, K, D, dt, n_steps, coupling, scheme=0, seed=1, omega=None, Kmat=None, phi=None,
         step0=0, M=100, samples=True):
    sde, ctx, dev = gpu
    om = torch.from_numpy(np.asarray(omega, dtype=np.float32)).to(dev)
    Kt = None if Kmat is None else torch.from_numpy(np.ascontiguousarray(Kmat, dtype=np.float32)).to(dev)
    if phi is None:
        ph = torch.empty((R, N), dtype=torch.float32, device=dev)
        init = sde.SDE_INIT_PHILOX
    else:
        ph = phi
        init = sde.SDE_INIT_FROM_STATE
    rs = torch.zeros((R, n_steps // M + 1), dtype=torch.float64, device=dev) if samples else None
    desc = sde.sde_kuramoto_desc(N, R, K, D, dt, n_steps, coupling, 0)
    run = sde.make_run(seed, step0=step0, scheme=scheme, init=init, sample_every=M, sync=1)
    sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, Kt, rs)
    return ph, rs


@pytest.mark.parametrize("scheme", [0, 1])
def test_meanfield_uniform_first_100_steps(gpu, scheme):
    """The uniform-coupling workload (N = 65536, omega ~ N(0,1), K = 3,
    D = 0.1, dt = 0.01, 16 realizations), first 100 steps, per oscillator."""
    cfg = sde_inputs.kuramoto_uniform()
    N, R = cfg["N"], cfg["R"]
    ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 0, scheme, cfg["seed"], cfg["omega"])
    ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD,
                                          scheme, cfg["seed"], cfg["omega"].astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"mean-field scheme {scheme}: max phase error {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_meanfield_order_parameter_trajectory(gpu):
    """r(t) every 100 steps over 2000 Heun steps at N = 8192, 8 realizations."""
    cfg = sde_inputs.kuramoto_uniform(N=8192, R=8)
    N, R = 8192, 8
    n = 2000
    _, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], n, 0, 0, cfg["seed"], cfg["omega"])
    _, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], n, 100, oracle.MEANFIELD, 0,
                                        cfg["seed"], cfg["omega"].astype(np.float64))
    d = rs.cpu().numpy() - rref
    se = d.std(ddof=1) / np.sqrt(d.size)
    print(f"r(t): max |diff| {np.abs(d).max():.2e}, mean {d.mean():.2e}, SE {se:.2e}")
    assert abs(d.mean()) <= 3 * se + 1e-4
    assert np.abs(d).max() <= 1e-3


@pytest.mark.parametrize("scheme", [0, 1])
def test_tiled_first_100_steps(gpu, scheme):
    """Alg. 3 (all N^2 sin terms) against the oracle's Eq. 3 sums, N = 3000
    (ragged against the 1024-oscillator tiles), 3 realizations."""
    N, R = 3000, 3
    rng = np.random.default_rng(4)
    omega = rng.standard_normal(N).astype(np.float32)
    ph, rs = _run(gpu, N, R, 3.0, 0.1, 0.01, 100, 1, scheme, 9, omega)
    ref, rref = oracle.kuramoto_integrate(N, R, 3.0, 0.1, 0.01, 100, 100, oracle.MEANFIELD, scheme, 9,
                                          omega.astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"tiled scheme {scheme}: max phase error {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_tiled_full_size_sampled(gpu):
    """The all-pairs sum at the uniform-coupling workload's own shape (N =
    65536, 16 realizations, one j slice, the tuned tile) for 20 Heun steps,
    realizations 0 and 15 against the oracle's Eq. 3 sums per oscillator."""
    sde, ctx, dev = gpu
    cfg = sde_inputs.kuramoto_uniform()
    N, R = cfg["N"], cfg["R"]
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_JSPLIT, 1)
    ph, rs = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], 20, 1, 0, cfg["seed"], cfg["omega"], M=10)
    st = sde.sde_get_stats(ctx)
    assert st["kura_jsplit"] == 1
    print(f"tiled full size: tile {st['kura_tile']} oscillators per lane", flush=True)
    got = ph.cpu().numpy()
    for r in (0, 15):
        ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 20, 10, oracle.MEANFIELD, 0,
                                              cfg["seed"], cfg["omega"].astype(np.float64), r_first=r, r_count=1)
        err = _circ_err(got[r], ref[0])
        print(f"tiled N = {N}, realization {r}: max phase error {err.max():.2e}")
        assert err.max() <= 1e-5
        np.testing.assert_allclose(rs.cpu().numpy()[r], rref[0], rtol=0, atol=1e-6)


def test_tiled_matches_meanfield_on_gpu(gpu):
    N, R = 4096, 2
    omega = sde_inputs.kuramoto_omega(N, 1.0, 3)
    a, ra = _run(gpu, N, R, 3.0, 0.1, 0.01, 200, 0, 0, 5, omega)
    b, rb = _run(gpu, N, R, 3.0, 0.1, 0.01, 200, 1, 0, 5, omega)
    d = a.cpu().numpy().astype(np.float64) - b.cpu().numpy()
    d = np.abs(np.mod(d + 0.5, 1.0) - 0.5) * 2 * np.pi
    assert d.max() <= 2e-5
    np.testing.assert_allclose(ra.cpu().numpy(), rb.cpu().numpy(), atol=1e-6)


@pytest.mark.parametrize("coupling,tol", [(2, 1e-5), (3, 1e-4), (4, 1e-5)])
def test_dense_first_100_steps(gpu, coupling, tol):
    """Dense heterogeneous K_ij (FP32, BF16x3, FP16x3 products): N = 520,
    R = 40 (both ragged against the 128-row / 32-realization tiles)."""
    N, R = 520, 40
    Kmat = sde_inputs.dense_coupling(N, 4.0, 11)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 12)
    ph, rs = _run(gpu, N, R, 4.0, 0.05, 0.005, 100, coupling, 0, 13, omega, Kmat)
    ref, rref = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, 100, 100, oracle.DENSE, 0, 13,
                                          omega.astype(np.float64), Kmat=Kmat.astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"dense coupling {coupling}: max phase error {err.max():.2e}, mean {err.mean():.2e}")
    assert err.max() <= tol
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=10 * tol)


@pytest.mark.parametrize("coupling,tol", [(2, 1e-5), (3, 1e-4), (4, 1e-5)])
@pytest.mark.parametrize("N,R,scheme", [(520, 40, 1), (1, 1, 0), (33, 3, 1), (200, 70, 0)])
def test_dense_euler_and_small_shapes(gpu, coupling, tol, N, R, scheme):
    """Euler-Maruyama (updated in place) and shapes below one 32-k block per
    wave of the split k loop: N = 1 (a lone oscillator: drift omega plus
    noise), N = 33 and 200 (2 and 7 k blocks), R = 70 (three realization
    tiles, the last ragged)."""
    Kmat = sde_inputs.dense_coupling(N, 4.0, 21)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 22)
    ph, rs = _run(gpu, N, R, 4.0, 0.05, 0.005, 100, coupling, scheme, 23, omega, Kmat)
    ref, rref = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, 100, 100, oracle.DENSE, scheme, 23,
                                          omega.astype(np.float64), Kmat=Kmat.astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"dense coupling {coupling}, N {N}, R {R}, scheme {scheme}: max phase error {err.max():.2e}")
    assert err.max() <= tol
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=10 * tol)


def test_dense_launch_choices(gpu):
    """Every dense launch choice, forced (8 or 4 waves splitting the k loop,
    row tiles in XCD bands or plain order; N = 1000 gives 8 row tiles, so
    the banding applies), for each product against the oracle over 50 Heun
    steps; the order of the tiles changes no arithmetic, so banded and plain
    runs of one wave count agree bit for bit."""
    sde, ctx, dev = gpu
    N, R, n = 1000, 40, 50
    Kmat = sde_inputs.dense_coupling(N, 4.0, 31)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 32)
    ref, _ = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, n, 0, oracle.DENSE, 0, 33,
                                       omega.astype(np.float64), Kmat=Kmat.astype(np.float64))
    for coupling, tol in [(2, 1e-5), (3, 1e-4), (4, 1e-5)]:
        got = {}
        for launch in range(1, 13):
            sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, launch)
            ph, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, coupling, 0, 33, omega, Kmat, samples=False)
            st = sde.sde_get_stats(ctx)
            waves = 4 if coupling == 2 or launch in (2, 4, 9, 10) else 8
            variant = 0 if coupling == 2 else {5: 1, 6: 1, 7: 2, 8: 2, 9: 3, 10: 3, 11: 4, 12: 4}.get(launch, 0)
            assert st["dense_waves"] == waves and st["dense_variant"] == variant
            assert st["dense_xcd_bands"] == (1 if launch in (1, 2, 5, 7, 9, 11) else 0)
            err = _circ_err(ph.cpu().numpy(), ref)
            print(f"dense coupling {coupling}, launch {launch}: max phase error {err.max():.2e}")
            assert err.max() <= tol
            got[launch] = ph.clone()
        assert torch.equal(got[1], got[3]) and torch.equal(got[2], got[4]) and torch.equal(got[5], got[6])
        assert torch.equal(got[7], got[8]) and torch.equal(got[9], got[10]) and torch.equal(got[11], got[12])
        if coupling == 2:
            assert all(torch.equal(got[1], got[k]) for k in (2, 5, 7, 9, 11))
    for bad in (-1, 13):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, bad)


@pytest.mark.parametrize("N,R", [(1000, 64), (100, 64), (40, 100), (3000, 40), (300, 70), (700, 9)])
def test_dense_two_halves(gpu, N, R):
    """The two-half launch (two workgroups per 128 x 32 tile over the two
    halves of k, A fragments shared through LDS by the wave pairs) against the
    oracle over 30 Heun steps: k extents of 32 blocks of 32, 4, 2 (some k
    slices idle) and 94 (halves of 47 blocks, slices of 12 and 11), and odd
    numbers of 32-realization tiles (R = 70 pads to 96: 3 tiles; R = 9: 1
    tile), where the launch falls back to the one-half kernel."""
    sde, ctx, dev = gpu
    n = 30
    Kmat = sde_inputs.dense_coupling(N, 4.0, 61)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 62)
    ref, _ = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, n, 0, oracle.DENSE, 0, 63,
                                       omega.astype(np.float64), Kmat=Kmat.astype(np.float64))
    even = ((R + 31) // 32) % 2 == 0
    for coupling, tol in [(3, 1e-4), (4, 1e-5)]:
        sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, 5)
        ph, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, coupling, 0, 63, omega, Kmat, samples=False)
        st = sde.sde_get_stats(ctx)
        assert st["dense_variant"] == (1 if even else 0) and st["dense_waves"] == 8
        err = _circ_err(ph.cpu().numpy(), ref)
        print(f"two halves N={N} R={R} coupling {coupling}: max phase error {err.max():.2e}", flush=True)
        assert err.max() <= tol
        # the same shapes through the wave-pair kernel (K shared through LDS)
        sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, 11)
        ph, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, coupling, 0, 63, omega, Kmat, samples=False)
        assert sde.sde_get_stats(ctx)["dense_variant"] == 4
        err = _circ_err(ph.cpu().numpy(), ref)
        print(f"wave pairs N={N} R={R} coupling {coupling}: max phase error {err.max():.2e}", flush=True)
        assert err.max() <= tol


@pytest.mark.parametrize("coupling,tol", [(2, 1e-5), (3, 1e-4), (4, 1e-5)])
def test_dense_against_direct_sum(gpu, coupling, tol):
    """The dense products against the oracle's plain double sum of Eq. 2,
    sum_j K_ij sin(phi_j - phi_i) per oscillator (not its Eq. 3 row form),
    over 20 Heun steps of 40 realizations of 300 oscillators."""
    sde, ctx, dev = gpu
    N, R, n = 300, 40, 20
    Kmat = sde_inputs.dense_coupling(N, 4.0, 71)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 72)
    ref, _ = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, n, 0, oracle.DIRECT, 0, 73,
                                       omega.astype(np.float64), Kmat=Kmat.astype(np.float64))
    ph, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, coupling, 0, 73, omega, Kmat, samples=False)
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"dense coupling {coupling} against the direct sum: max phase error {err.max():.2e}")
    assert err.max() <= tol


def test_dense_tuner(gpu):
    """Left to the tuner, the first call of a shape class times the launch
    choices and caches one; the next call reuses it without tuning and
    equals, bit for bit, a run forced to that choice."""
    sde, ctx, dev = gpu
    N, R, n = 2000, 9, 10
    Kmat = sde_inputs.dense_coupling(N, 4.0, 51)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 52)
    _run(gpu, N, R, 4.0, 0.05, 0.005, n, 3, 0, 53, omega, Kmat, samples=False)
    st1 = sde.sde_get_stats(ctx)
    assert st1["tuned"] == 1 and st1["dense_waves"] in (4, 8) and st1["dense_xcd_bands"] in (0, 1)
    a, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, 3, 0, 53, omega, Kmat, samples=False)
    st2 = sde.sde_get_stats(ctx)
    assert st2["tuned"] == 0
    chosen = (st1["dense_variant"], st1["dense_waves"], st1["dense_xcd_bands"])
    assert (st2["dense_variant"], st2["dense_waves"], st2["dense_xcd_bands"]) == chosen
    # the forced launch of the same kernel, wave count and tile order
    launch = {(0, 8, 1): 1, (0, 4, 1): 2, (0, 8, 0): 3, (0, 4, 0): 4, (1, 8, 1): 5, (1, 8, 0): 6,
              (2, 8, 1): 7, (2, 8, 0): 8, (3, 4, 1): 9, (3, 4, 0): 10, (4, 8, 1): 11, (4, 8, 0): 12}[chosen]
    sde.sde_set_option(ctx, sde.SDE_OPT_DENSE_LAUNCH, launch)
    b, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, 3, 0, 53, omega, Kmat, samples=False)
    assert torch.equal(a, b)
    print(f"dense tuner: kernel {st1['dense_variant']}, {st1['dense_waves']} waves, "
          f"bands {st1['dense_xcd_bands']} ({st1['tune_ms']:.2f} ms)")


def test_dense_full_size_sampled(gpu):
    """The dense workload at its size -- N = 4096, 256 realizations, the
    BF16x3 product -- for 200 steps, realizations 0..3 checked against the
    oracle (which draws the same keyed noise)."""
    cfg = sde_inputs.kuramoto_dense()
    N, R = cfg["N"], cfg["R"]
    n = 200
    ph, _ = _run(gpu, N, R, cfg["K"], cfg["D"], cfg["dt"], n, 3, 0, cfg["seed"], cfg["omega"], cfg["Kmat"])
    ref, _ = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], n, 0, oracle.DENSE, 0, cfg["seed"],
                                       cfg["omega"].astype(np.float64), Kmat=cfg["Kmat"].astype(np.float64),
                                       r_first=0, r_count=4)
    err = _circ_err(ph.cpu().numpy()[:4], ref)
    print(f"dense bf16x3 at N=4096, R=256, 200 steps: max phase error {err.max():.2e}")
    assert err.max() <= 2e-4


@pytest.mark.parametrize("coupling,tol", [(2, 1e-5), (3, 2e-5), (4, 1e-5)])
def test_dense_twice_the_benchmark_size_sampled(gpu, coupling, tol):
    """N = 8192 (32 k blocks per wave of the split loop), R = 32, 20 Heun
    steps; realizations 0 and 1 against the oracle.  BF16x3 bound: the drift
    error bound 1.5 K 2^-15 per unit time (independent of N: a row of K sums
    to at most 1.5 K) over 20 steps of dt = 0.005, 1.8e-5."""
    N, R, n = 8192, 32, 20
    Kmat = sde_inputs.dense_coupling(N, 4.0, 41)
    omega = sde_inputs.kuramoto_omega(N, 0.5, 42)
    ph, _ = _run(gpu, N, R, 4.0, 0.05, 0.005, n, coupling, 0, 43, omega, Kmat, samples=False)
    ref, _ = oracle.kuramoto_integrate(N, R, 4.0, 0.05, 0.005, n, 0, oracle.DENSE, 0, 43,
                                       omega.astype(np.float64), Kmat=Kmat.astype(np.float64), r_first=0, r_count=2)
    err = _circ_err(ph.cpu().numpy()[:2], ref)
    print(f"dense coupling {coupling} at N = 8192: max phase error {err.max():.2e}")
    assert err.max() <= tol


def test_dense_uniform_matrix_equals_meanfield(gpu):
    """K_ij = K/N off the diagonal (zero diagonal) is the uniform model."""
    N, R = 1024, 32
    K = 2.5
    Kmat = np.full((N, N), K / N, dtype=np.float32)
    np.fill_diagonal(Kmat, 0.0)
    omega = sde_inputs.kuramoto_omega(N, 1.0, 7)
    a, _ = _run(gpu, N, R, K, 0.1, 0.01, 100, 2, 0, 3, omega, Kmat)
    b, _ = _run(gpu, N, R, K, 0.1, 0.01, 100, 0, 0, 3, omega)
    d = a.cpu().numpy().astype(np.float64) - b.cpu().numpy()
    d = np.abs(np.mod(d + 0.5, 1.0) - 0.5) * 2 * np.pi
    assert d.max() <= 2e-5


@pytest.mark.parametrize("coupling,N", [(0, 65536), (1, 2048)])
def test_identical_oscillator_threshold(gpu, coupling, N):
    """omega = 0: stationary r solves r = I1(K r/D)/I0(K r/D) above K_c = 2D
    (0.8315 at K/D = 4) and is O(N^-1/2) below it (K/D = 1)."""
    D = 0.25
    R = 2
    n = 3000 if coupling == 1 else 6000
    tol = 0.03 if N < 10000 else 0.02
    omega = np.zeros(N, dtype=np.float32)
    for KD, lo, hi in [(4.0, 0.8315 - tol, 0.8315 + tol), (1.0, 0.0, 0.08)]:
        _, rs = _run(gpu, N, R, KD * D, D, 0.01, n, coupling, 0, 17, omega)
        r_late = rs.cpu().numpy()[:, -10:].mean()
        print(f"coupling {coupling}, K/D = {KD}: late r = {r_late:.4f}")
        assert lo <= r_late <= hi


@pytest.mark.parametrize("coupling", [0, 1, 3])
def test_resume_bit_identical(gpu, coupling):
    sde, ctx, dev = gpu
    N, R = 1000, 32
    omega = sde_inputs.kuramoto_omega(N, 1.0, 2)
    Kmat = sde_inputs.dense_coupling(N, 3.0, 2) if coupling >= 2 else None
    full, _ = _run(gpu, N, R, 3.0, 0.1, 0.01, 50, coupling, 0, 8, omega, Kmat, samples=False)
    a, _ = _run(gpu, N, R, 3.0, 0.1, 0.01, 21, coupling, 0, 8, omega, Kmat, samples=False)
    b, _ = _run(gpu, N, R, 3.0, 0.1, 0.01, 29, coupling, 0, 8, omega, Kmat, phi=a, step0=21, samples=False)
    assert torch.equal(full, b)


def test_deterministic_meanfield(gpu):
    cfg = sde_inputs.kuramoto_uniform()
    a, ra = _run(gpu, cfg["N"], cfg["R"], cfg["K"], cfg["D"], cfg["dt"], 300, 0, 0, 4, cfg["omega"])
    b, rb = _run(gpu, cfg["N"], cfg["R"], cfg["K"], cfg["D"], cfg["dt"], 300, 0, 0, 4, cfg["omega"])
    assert torch.equal(a, b) and torch.equal(ra, rb)


def test_kuramoto_invalid_arguments(gpu):
    sde, ctx, dev = gpu
    N, R = 64, 2
    ph = torch.zeros((R, N), dtype=torch.float32, device=dev)
    om = torch.zeros(N, dtype=torch.float32, device=dev)
    Km = torch.zeros((N, N), dtype=torch.float32, device=dev)
    run = sde.make_run(1, sync=1)
    bad = [(sde.sde_kuramoto_desc(0, R, 1.0, 0.1, 0.01, 10, 0, 0), None),
           (sde.sde_kuramoto_desc(N, 0, 1.0, 0.1, 0.01, 10, 0, 0), None),
           (sde.sde_kuramoto_desc(N, R, 1.0, 0.1, 0.0, 10, 0, 0), None),
           (sde.sde_kuramoto_desc(N, R, 1.0, -0.1, 0.01, 10, 0, 0), None),
           (sde.sde_kuramoto_desc(N, R, float("nan"), 0.1, 0.01, 10, 0, 0), None),
           (sde.sde_kuramoto_desc(N, R, 1.0, 0.1, 0.01, 10, 3, 0), None),
           (sde.sde_kuramoto_desc(N, R, 1.0, 0.1, 0.01, 10, 0, 0), Km),
           (sde.sde_kuramoto_desc(N, R, 1.0, 0.1, 0.01, 10, 9, 0), None)]
    for desc, K in bad:
        with pytest.raises(sde.SDEError) as e:
            sde.sde_kuramoto_integrate(ctx, desc, run, ph, om, K)
        assert e.value.status == sde.SDE_ERR_INVALID
    assert torch.count_nonzero(ph) == 0
