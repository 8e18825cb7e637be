"""Pins of the oracle's integrators against closed forms (CPU only).

Each check is chosen so that a plausible slip in the oracle (a dropped term,
a wrong sign, noise in the wrong place, the second drift evaluated at the
wrong time) fails at least one of them:
  * OU: the exact stationary variance of the discrete Heun and Euler
    recursions and the exact decay of the mean (step structure, noise
    placement, weak order);
  * free diffusion: Var = 2 D t exactly (noise amplitude);
  * Josephson junction at a = f = 0: Boltzmann equilibrium <v^2> = D/m and
    <cos phi> = I1(1/D)/I0(1/D) (drift sign, friction, inertia, noise);
  * overdamped tilted washboard: v = sqrt(f^2 - 1)/gamma (bias, friction);
  * noise-free driven junction: global error of order dt^2 against a
    high-order library integrator (drive term and its time argument);
  * Kuramoto: Adler's law for N = 2, the identical-oscillator
    self-consistency r = I1(K r/D)/I0(K r/D) with K_c = 2D (coupling sign and
    scale), and the Eq. 3 identity between the coupling forms.
"""
import numpy as np
import pytest
from scipy import integrate, optimize, special

import sde_inputs

HEUN, EULER = 0, 1


# ---------------------------------------------------------------- OU ------
def _ou_discrete_var(scheme, k, D, dt):
    h = k * dt
    s2 = 2 * D * dt
    if scheme == HEUN:
        a = 1 - h + h * h / 2
        return s2 * (1 - h / 2) ** 2 / (1 - a * a)
    a = 1 - h
    return s2 / (1 - a * a)


@pytest.mark.parametrize("scheme", [HEUN, EULER])
@pytest.mark.parametrize("h", [0.4, 0.2])
def test_ou_discrete_stationary_variance(orc, scheme, h):
    k, D = 1.0, 0.5
    n_paths = 200_000
    n_steps = int(round(25.0 / h))
    x = orc.ou_integrate(k, D, h / k, n_steps, scheme, 4242, np.zeros(n_paths))
    var = x.var()
    exact = _ou_discrete_var(scheme, k, D, h / k)
    se = exact * np.sqrt(2.0 / n_paths)
    assert abs(var - exact) < 4 * se
    # the discretisation bias is resolved: Heun -4.76% / -1.10%, Euler +25% / +11.1%
    cont = D / k
    assert abs(var - cont) > 4 * se


def test_ou_weak_order_of_bias():
    """Closed forms of the bias give slope 2 (Heun) and 1 (Euler)."""
    k, D = 1.0, 1.0
    for scheme, order in [(HEUN, 2), (EULER, 1)]:
        b = [abs(_ou_discrete_var(scheme, k, D, h) / (D / k) - 1) for h in (0.1, 0.05, 0.025)]
        slopes = np.log2(np.array(b[:-1]) / np.array(b[1:]))
        assert np.all(np.abs(slopes - order) < 0.1)
    # the tabulated relative errors of Heun's stationary variance
    rel = [_ou_discrete_var(HEUN, 1.0, 1.0, h) - 1 for h in (0.4, 0.2, 0.1, 0.05)]
    np.testing.assert_allclose(rel, [-0.0476, -0.0110, -0.00262, -0.00064], atol=6e-5)


def test_ou_mean_decay(orc):
    """With noise the mean still follows the deterministic recursion exactly."""
    k, D, dt, n = 2.0, 0.3, 0.05, 40
    x = orc.ou_integrate(k, D, dt, n, HEUN, 7, np.ones(100_000))
    h = k * dt
    mean_exact = (1 - h + h * h / 2) ** n
    var_exact = sum((2 * D * dt) * (1 - h / 2) ** 2 * (1 - h + h * h / 2) ** (2 * j) for j in range(n))
    assert abs(x.mean() - mean_exact) < 4 * np.sqrt(var_exact / x.size)
    # the continuum value e^{-k t} agrees to O(h^2) per unit time
    assert abs(mean_exact - np.exp(-k * dt * n)) < 2e-3


def test_ou_noise_free_is_deterministic(orc):
    x = orc.ou_integrate(1.0, 0.0, 0.1, 10, HEUN, 1, np.full(3, 2.0))
    np.testing.assert_allclose(x, 2.0 * (1 - 0.1 + 0.005) ** 10, rtol=1e-14)


# ----------------------------------------------------- free diffusion -----
@pytest.mark.parametrize("scheme", [HEUN, EULER])
def test_free_diffusion_variance(orc, scheme):
    N, D, dt, n = 40_000, 0.7, 0.01, 150
    phi0 = np.zeros((1, N))
    phi, _ = orc.kuramoto_integrate(N, 1, 0.0, D, dt, n, 0, orc.MEANFIELD, scheme, 11,
                                    np.zeros(N), phi0=phi0)
    t = n * dt
    var = phi.var()
    assert abs(var - 2 * D * t) < 4 * 2 * D * t * np.sqrt(2.0 / N)
    assert abs(phi.mean()) < 4 * np.sqrt(2 * D * t / N)


# ------------------------------------------------ Josephson junction ------
def _jj(**kw):
    return sde_inputs.jj_point(**kw)


@pytest.mark.parametrize("D", [0.5, 1.0])
def test_jj_boltzmann_equilibrium(orc, D):
    """a = f = 0: stationary density exp(-(v^2/2 - cos phi)/D)."""
    n_paths = 16384
    pt = _jj(m=1.0, gamma=1.0, a=0.0, omega=2 * np.pi, f=0.0, D=D, n_paths=n_paths,
             steps_per_period=100, n_steps=3000, n_transient=0)
    res = orc.jj_integrate([pt], seed=77)
    v, phi = res["v"], res["phi"]
    v2 = (v ** 2).mean()
    assert abs(v2 - D) < 4 * D * np.sqrt(2.0 / n_paths) + 2e-3
    c = np.cos(phi)
    expect = special.i1(1 / D) / special.i0(1 / D)
    assert abs(c.mean() - expect) < 4 * c.std() / np.sqrt(n_paths) + 2e-3
    assert abs(v.mean()) < 4 * np.sqrt(D / n_paths)


@pytest.mark.parametrize("f,gamma", [(1.5, 0.8), (2.5, 1.3), (0.6, 1.0)])
def test_jj_overdamped_washboard_velocity(orc, f, gamma):
    """m = 0, D = 0, a = 0: v = sqrt(f^2 - 1)/gamma above f = 1, else 0."""
    n_steps, S = 200_000, 100
    pt = _jj(m=0.0, gamma=gamma, a=0.0, omega=2 * np.pi, f=f, D=0.0, n_paths=4,
             steps_per_period=S, n_steps=n_steps, n_transient=1000)
    res = orc.jj_integrate([pt], seed=1)
    vbar = res["point_sums"][0, 0] / 4
    T = (n_steps - 1000) * (1.0 / S)
    exact = np.sqrt(f * f - 1) / gamma if f > 1 else 0.0
    assert abs(vbar - exact) < 2 * np.pi / T + 1e-4


def _jj_rhs(t, y, p):
    phi, v = y
    return [v, (-np.sin(phi) - p["gamma"] * v + p["a"] * np.cos(p["omega"] * t) + p["f"]) / p["m"]]


def test_jj_deterministic_order_two(orc):
    """D = 0 with the drive on: Heun's global error falls as dt^2."""
    p = dict(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=0.1)
    T_end = 4 * 2 * np.pi / 4.9
    y0 = [0.3, -0.7]
    ref = integrate.solve_ivp(_jj_rhs, (0, T_end), y0, args=(p,), method="DOP853",
                              rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for S in (50, 100, 200, 400):
        pt = _jj(D=0.0, n_paths=1, steps_per_period=S, n_steps=4 * S, **p)
        res = orc.jj_integrate([pt], seed=0, state=(np.array([y0[0]]), np.array([y0[1]]),
                                                    np.zeros(1)))
        errs.append(np.hypot(res["phi"][0] - ref[0], res["v"][0] - ref[1]))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.2), (errs, slopes)
    assert errs[-1] < 1e-4


def test_jj_euler_order_one(orc):
    p = dict(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=0.1)
    T_end = 2 * 2 * np.pi / 4.9
    y0 = [0.3, -0.7]
    ref = integrate.solve_ivp(_jj_rhs, (0, T_end), y0, args=(p,), method="DOP853",
                              rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for S in (200, 400, 800):
        pt = _jj(D=0.0, n_paths=1, steps_per_period=S, n_steps=2 * S, **p)
        res = orc.jj_integrate([pt], seed=0, scheme=EULER,
                               state=(np.array([y0[0]]), np.array([y0[1]]), np.zeros(1)))
        errs.append(np.hypot(res["phi"][0] - ref[0], res["v"][0] - ref[1]))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 1) < 0.2), (errs, slopes)


# ---- the paper's own potential V(x) = sin(2 pi x), x in periods (Sec. 3) ----
P2 = sde_inputs.POT_SIN2PI


@pytest.mark.parametrize("D", [0.5, 1.0])
def test_jj_sin2pi_boltzmann_equilibrium(orc, D):
    """a = f = 0: stationary density exp(-(v^2/2 + sin 2 pi x)/D), so
    <v^2> = D, <sin 2 pi x> = -I1(1/D)/I0(1/D) and <cos 2 pi x> = 0.  A wrong
    sign of the force flips the sin moment; a missing 2 pi factor changes it
    to the moment of a potential 2 pi times shallower."""
    n_paths = 16384
    pt = _jj(m=1.0, gamma=1.0, a=0.0, omega=2 * np.pi, f=0.0, D=D, n_paths=n_paths,
             steps_per_period=400, n_steps=12000, n_transient=0, potential=P2)
    res = orc.jj_integrate([pt], seed=78)
    v, x = res["v"], res["phi"]
    assert abs((v ** 2).mean() - D) < 4 * D * np.sqrt(2.0 / n_paths) + 4e-3
    s_, c_ = np.sin(2 * np.pi * x), np.cos(2 * np.pi * x)
    expect = -special.i1(1 / D) / special.i0(1 / D)
    assert abs(s_.mean() - expect) < 4 * s_.std() / np.sqrt(n_paths) + 2e-3
    assert abs(c_.mean()) < 4 * c_.std() / np.sqrt(n_paths) + 2e-3
    wrong = -special.i1(1 / (2 * np.pi * D)) / special.i0(1 / (2 * np.pi * D))
    assert abs(s_.mean() - wrong) > 0.1


@pytest.mark.parametrize("f,gamma", [(7.5, 0.8), (9.0, 1.3), (5.0, 1.0)])
def test_jj_sin2pi_overdamped_washboard_velocity(orc, f, gamma):
    """m = 0, D = 0, a = 0: gamma x' = f - 2 pi cos 2 pi x runs with
    v = 1 / int_0^1 gamma dx / (f - 2 pi cos 2 pi x) = sqrt(f^2 - 4 pi^2)/gamma
    above f = 2 pi and is locked (v = 0) below."""
    n_steps, S = 200_000, 400
    pt = _jj(m=0.0, gamma=gamma, a=0.0, omega=2 * np.pi, f=f, D=0.0, n_paths=4,
             steps_per_period=S, n_steps=n_steps, n_transient=1000, potential=P2)
    res = orc.jj_integrate([pt], seed=1)
    vbar = res["point_sums"][0, 0] / 4
    T = (n_steps - 1000) * (1.0 / S)
    exact = np.sqrt(f * f - 4 * np.pi ** 2) / gamma if f > 2 * np.pi else 0.0
    assert abs(vbar - exact) < 1.0 / T + 1e-3 * max(exact, 1.0)


def _sin2pi_rhs(t, y, p):
    x, v = y
    return [v, (-2 * np.pi * np.cos(2 * np.pi * x) - p["gamma"] * v + p["a"] * np.cos(p["omega"] * t)
                + p["f"]) / p["m"]]


def test_jj_sin2pi_deterministic_order_two(orc):
    """D = 0 with the paper's drive (a = 4.2, omega = 4.9, gamma = 0.9,
    f = 0.1): Heun's global error against a high-order solution falls as dt^2."""
    p = dict(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=0.1)
    T_end = 2 * 2 * np.pi / 4.9
    y0 = [0.3, -0.7]
    ref = integrate.solve_ivp(_sin2pi_rhs, (0, T_end), y0, args=(p,), method="DOP853",
                              rtol=1e-13, atol=1e-13).y[:, -1]
    errs = []
    for S in (100, 200, 400, 800):
        pt = _jj(D=0.0, n_paths=1, steps_per_period=S, n_steps=2 * S, potential=P2, **p)
        res = orc.jj_integrate([pt], seed=0, state=(np.array([y0[0]]), np.array([y0[1]]),
                                                    np.zeros(1)))
        errs.append(np.hypot(res["phi"][0] - ref[0], res["v"][0] - ref[1]))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.2), (errs, slopes)
    assert errs[-1] < 1e-3


def test_jj_sin2pi_absolute_negative_mobility(orc):
    """The Fig. 2 parameters (a = 4.2, gamma = 0.9, omega = 4.9, D = 0.001)
    lie in the anomalous-response regime the paper names (Sec. 3): a small
    bias f = +0.1 drives a negative mean velocity, f = -0.1 a positive one,
    each more than 5 standard errors from zero (512 paths, 100 periods of
    transient, 300 averaged).  Only the sign is pinned; the magnitude still
    drifts over the paper's 2000 periods."""
    out = {}
    for f in (0.1, -0.1):
        pt = _jj(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=f, D=1e-3, n_paths=512, steps_per_period=100,
                 n_steps=100 * 400, n_transient=100 * 100, potential=P2)
        r = orc.jj_integrate([pt], seed=11)
        vb = r["acc"] / (pt["n_steps"] - pt["n_transient"])
        out[f] = (vb.mean(), vb.std(ddof=1) / np.sqrt(vb.size))
    assert out[0.1][0] < -5 * out[0.1][1], out
    assert out[-0.1][0] > 5 * out[-0.1][1], out


def test_jj_sin2pi_initial_conditions(orc):
    """x0 = U(x0) in periods (no 2 pi), v0 = -2 + 4 U(x1)."""
    import oracle.philox_ref as pref
    pt = sde_inputs.jj_point(n_paths=6, n_steps=0, potential=P2)
    res = orc.jj_integrate([pt], seed=4)
    for p in range(6):
        w = pref.block(4, 1, p, 0, 0)
        assert res["phi"][p] == (w[0] >> 8) / 2**24
        assert res["v"][p] == -2 + 4 * ((w[1] >> 8) / 2**24)


def test_jj_potentials_mix_in_one_call(orc):
    """Each point follows its own potential; a batch equals the points run
    alone (same point ids)."""
    pts = [sde_inputs.jj_point(n_paths=5, n_steps=50, potential=k) for k in (0, 1, 0)]
    both = orc.jj_integrate(pts, seed=6)
    off = 0
    for q, pt in enumerate(pts):
        alone = orc.jj_integrate([pt], seed=6, point_ids=[q])
        np.testing.assert_array_equal(both["phi"][off:off + 5], alone["phi"])
        off += 5
    assert not np.allclose(both["phi"][:5], both["phi"][5:10])


def test_jj_resume_is_bit_identical(orc):
    pts = sde_inputs.jj_single(n_paths=64, n_steps=300)
    full = orc.jj_integrate(pts, seed=5)
    a = orc.jj_integrate([dict(pts[0], n_steps=123)], seed=5)
    b = orc.jj_integrate([dict(pts[0], n_steps=177)], seed=5, step0=123,
                         state=(a["phi"], a["v"], a["acc"]))
    for k in ("phi", "v", "acc"):
        assert np.array_equal(full[k], b[k])
    assert np.array_equal(full["point_sums"], b["point_sums"])


def test_jj_initial_conditions(orc):
    """phi0 ~ U[0, 2pi) and v0 ~ U[-2, 2] from the INIT stream, path p of point q."""
    import oracle.philox_ref as pref
    pts = [sde_inputs.jj_point(n_paths=8, n_steps=1), sde_inputs.jj_point(n_paths=5, n_steps=1)]
    res = orc.jj_integrate([dict(p, n_steps=0) for p in pts], seed=3, n_record=0)
    for q, off in [(0, 0), (1, 8)]:
        for p in range(pts[q]["n_paths"]):
            w = pref.block(3, 1, p, q, 0)
            assert res["phi"][off + p] == 2 * np.pi * ((w[0] >> 8) / 2**24)
            assert res["v"][off + p] == -2 + 4 * ((w[1] >> 8) / 2**24)


def test_jj_point_sums_definition(orc):
    pts = [sde_inputs.jj_point(n_paths=16, n_steps=200, n_transient=50)]
    res = orc.jj_integrate(pts, seed=9, n_record=200)
    vbar = res["rec_v"][50:].mean(axis=0)
    np.testing.assert_allclose(res["point_sums"][0], [vbar.sum(), (vbar ** 2).sum()], rtol=1e-12)


def test_jj_invalid_arguments(orc):
    bad = [dict(sde_inputs.jj_point(), gamma=-1.0), dict(sde_inputs.jj_point(), n_paths=0),
           dict(sde_inputs.jj_point(), steps_per_period=0), dict(sde_inputs.jj_point(), D=np.nan)]
    for p in bad:
        with pytest.raises(ValueError):
            orc.jj_integrate([p], seed=1)


# ---------------------------------------------------------- Kuramoto -----
def test_kuramoto_adler_drifting(orc):
    """N = 2, K_ij = K/2: psi = phi2 - phi1 obeys psi' = dw - K sin psi."""
    K, dw, dt, n = 1.0, 2.0, 0.01, 200_000
    omega = np.array([-dw / 2, dw / 2])
    phi, _ = orc.kuramoto_integrate(2, 1, K, 0.0, dt, n, 0, orc.DIRECT, HEUN, 1, omega,
                                    phi0=np.zeros((1, 2)))
    rate = (phi[0, 1] - phi[0, 0]) / (n * dt)
    assert abs(rate - np.sqrt(dw * dw - K * K)) < 2 * np.pi / (n * dt) + 1e-4


def test_kuramoto_adler_locked(orc):
    K, dw = 1.0, 0.5
    omega = np.array([-dw / 2, dw / 2])
    phi, _ = orc.kuramoto_integrate(2, 1, K, 0.0, 0.01, 5000, 0, orc.MEANFIELD, HEUN, 1, omega,
                                    phi0=np.array([[0.0, 2.0]]))
    psi = np.mod(phi[0, 1] - phi[0, 0] + np.pi, 2 * np.pi) - np.pi
    assert abs(psi - np.arcsin(dw / K)) < 1e-8


def _r_selfconsistent(KD):
    if KD <= 2:
        return 0.0
    return optimize.brentq(lambda r: special.i1(KD * r) / special.i0(KD * r) - r, 1e-6, 1.0)


def test_selfconsistency_values():
    """r = I1(K r/D)/I0(K r/D): 0.5897, 0.7242, 0.8315, 0.9455 at K/D = 2.5, 3, 4, 10."""
    got = [_r_selfconsistent(x) for x in (2.5, 3.0, 4.0, 10.0)]
    np.testing.assert_allclose(got, [0.5897, 0.7242, 0.8315, 0.9455], atol=2e-4)


@pytest.mark.parametrize("KD", [1.0, 4.0, 10.0])
def test_kuramoto_identical_threshold(orc, KD):
    """omega = 0: the stationary order parameter solves the self-consistency
    equation; below K_c = 2D it is O(N^-1/2)."""
    N, D, dt = 4096, 0.25, 0.01
    K = KD * D
    n, M = 6000, 100
    phi, rs = orc.kuramoto_integrate(N, 1, K, D, dt, n, M, orc.MEANFIELD, HEUN, 21, np.zeros(N))
    r_late = rs[0, 30:].mean()
    expect = _r_selfconsistent(KD)
    if KD > 2:
        assert abs(r_late - expect) < 0.012
    else:
        assert r_late < 0.06


def test_kuramoto_repulsive_desynchronises(orc):
    """A flipped coupling sign gives r -> O(N^-1/2) even from a synchronised start."""
    N = 4096
    phi, rs = orc.kuramoto_integrate(N, 1, -1.0, 0.25, 0.01, 3000, 100, orc.MEANFIELD, HEUN, 3,
                                     np.zeros(N), phi0=np.zeros((1, N)))
    assert rs[0, 0] == pytest.approx(1.0)
    assert rs[0, -5:].mean() < 0.06


def test_eq3_identity_between_coupling_forms(orc):
    rng = np.random.default_rng(0)
    N, K = 700, 2.7
    phi = rng.uniform(-20, 20, N)
    omega = rng.standard_normal(N)
    mf = orc.kuramoto_rhs(phi, omega, K, orc.MEANFIELD)
    direct = orc.kuramoto_rhs(phi, omega, K, orc.DIRECT)
    np.testing.assert_allclose(mf, direct, rtol=0, atol=1e-12 * N * K / N + 1e-12)
    # dense with K_ij = K/N off the diagonal equals the uniform sums (the
    # diagonal term is sin 0 = 0)
    Kmat = np.full((N, N), K / N)
    np.fill_diagonal(Kmat, 0.0)
    dense = orc.kuramoto_rhs(phi, omega, K, orc.DENSE, Kmat)
    np.testing.assert_allclose(dense, direct, rtol=0, atol=1e-12)
    # heterogeneous K: the Eq. 3 row form equals the double sum of Eq. 2
    Kh = sde_inputs.dense_coupling(N, 4.0, 5).astype(np.float64)
    dense_h = orc.kuramoto_rhs(phi, omega, K, orc.DENSE, Kh)
    direct_h = orc.kuramoto_rhs(phi, omega, K, orc.DIRECT, Kh)
    np.testing.assert_allclose(dense_h, direct_h, rtol=0, atol=1e-12)
    # and a hand-written double loop on a few rows
    for i in (0, 13, N - 1):
        ref = omega[i] + sum(Kh[i, j] * np.sin(phi[j] - phi[i]) for j in range(N))
        assert abs(dense_h[i] - ref) < 1e-12


def test_kuramoto_order_parameter_definition(orc):
    N = 257
    omega = np.zeros(N)
    phi, rs = orc.kuramoto_integrate(N, 3, 1.0, 0.1, 0.01, 0, 1, orc.MEANFIELD, HEUN, 8, omega,
                                     r_first=1, r_count=2)
    for k in range(2):
        assert rs[k, 0] == pytest.approx(abs(np.exp(1j * phi[k]).mean()), abs=1e-14)


def test_kuramoto_initial_phases(orc):
    import oracle.philox_ref as pref
    N = 5
    phi, _ = orc.kuramoto_integrate(N, 4, 1.0, 0.1, 0.01, 0, 0, orc.MEANFIELD, HEUN, 8,
                                    np.zeros(N), r_first=2, r_count=2)
    for rr in range(2):
        for i in range(N):
            w = pref.block(8, 1, i, 2 + rr, 0)
            assert phi[rr, i] == 2 * np.pi * ((w[0] >> 8) / 2**24)


def test_kuramoto_noise_stream(orc):
    """With K = 0 one Euler step adds omega dt + sqrt(2 D dt) G(NOISE, i, r, n)."""
    N, D, dt = 6, 0.3, 0.02
    omega = np.arange(N, dtype=np.float64)
    phi0 = np.zeros((1, N))
    phi, _ = orc.kuramoto_integrate(N, 3, 0.0, D, dt, 1, 0, orc.MEANFIELD, EULER, 4, omega,
                                    phi0=phi0, step0=6, r_first=2, r_count=1)
    for i in range(N):
        g = orc.gauss(4, 0, i, 2, 6)
        assert phi[0, i] == pytest.approx(omega[i] * dt + np.sqrt(2 * D * dt) * g, abs=1e-15)
