"""Pins of the oracle's overdamped (m = 0) branch with noise (CPU only).

Eq. 1 without inertia reads gamma x' = -V'(x) + a cos(w t) + f
+ sqrt(2 gamma D) xi(t), i.e. x' = (...)/gamma + sqrt(2 D/gamma) xi: both the
drift and the noise carry the friction, in different powers.  Two facts fix
them independently of the oracle:

  * Boltzmann equilibrium at a = f = 0: the stationary density is
    exp(-V(x)/D) whatever gamma is, so <cos phi> = I1(1/D)/I0(1/D) for
    V = -cos phi and <sin 2 pi x> = -I1(1/D)/I0(1/D) for V = sin 2 pi x.  A
    noise amplitude with the wrong power of gamma equilibrates at the
    temperature D gamma^k instead and moves the moment.
  * Relaxation from the bottom of a well at small D: the linearised motion
    x' = -(V''/gamma) x + sqrt(2 D/gamma) xi is an OU process, and the
    variance after n steps of the discrete Heun (or Euler) recursion has a
    closed form in h = V'' dt/gamma and s^2 = 2 D dt/gamma.  It resolves the
    1/gamma of the drift (through h) and of the noise (through s^2).

The last test compiles copies of the oracle with the overdamped noise or
drift written wrongly and checks that these pins reject every copy.
"""
import os

import numpy as np
import pytest
from scipy import special

import sde_inputs

HEUN, EULER = 0, 1
P1, P2 = sde_inputs.POT_SIN, sde_inputs.POT_SIN2PI


def _pt(**kw):
    return sde_inputs.jj_point(**kw)


def check_boltzmann(orc, pot, gamma, D=0.5, n_paths=16384):
    """a = f = 0, m = 0: the stationary moment of the potential's shape."""
    if pot == P1:
        S, n_steps = 100, 3000          # dt = 0.01, t = 30 >= 12 relaxation times
    else:
        S, n_steps = 1000, 20000        # dt = 1e-3 (V'' dt/gamma <= 0.1), t = 20
    pt = _pt(m=0.0, gamma=gamma, a=0.0, omega=2 * np.pi, f=0.0, D=D, n_paths=n_paths,
             steps_per_period=S, n_steps=n_steps, n_transient=0, potential=pot)
    x = orc.jj_integrate([pt], seed=91)["phi"]
    moment = np.cos(x) if pot == P1 else np.sin(2 * np.pi * x)
    expect = special.i1(1 / D) / special.i0(1 / D) * (1 if pot == P1 else -1)
    tol = 4 * moment.std() / np.sqrt(n_paths) + 2e-3
    assert abs(moment.mean() - expect) < tol, (moment.mean(), expect, tol)
    return moment.mean()


def _ou_var(scheme, h, s2, n):
    """Variance after n steps of x' = x a + s psi b from x = 0: Heun has
    a = 1 - h + h^2/2, b = 1 - h/2 (the predictor's noise enters the second
    drift evaluation); Euler a = 1 - h, b = 1."""
    a, b = (1 - h + h * h / 2, 1 - h / 2) if scheme == HEUN else (1 - h, 1.0)
    return s2 * b * b * (1 - a ** (2 * n)) / (1 - a * a)


def check_relaxation(orc, pot, gamma, scheme, D=1e-4, n_paths=40000):
    """All paths start at the bottom of a well (phi = 0 for -sin phi,
    x = 3/4 for sin 2 pi x) and relax for kt = 1/2, k = V''/gamma."""
    if pot == P1:
        x0, curv, S = 0.0, 1.0, 100
    else:
        x0, curv, S = 0.75, 4 * np.pi ** 2, 10000
    dt = 1.0 / S                           # omega = 2 pi: one time unit per drive period
    k = curv / gamma
    n = max(1, int(round(0.5 / (k * dt))))
    pt = _pt(m=0.0, gamma=gamma, a=0.0, omega=2 * np.pi, f=0.0, D=D, n_paths=n_paths,
             steps_per_period=S, n_steps=n, n_transient=0, potential=pot)
    state = (np.full(n_paths, x0), np.zeros(n_paths), np.zeros(n_paths))
    x = orc.jj_integrate([pt], seed=92, scheme=scheme, state=state)["phi"] - x0
    s2 = 2 * D * dt / gamma                # x in its own units: radians or periods
    exact = _ou_var(scheme, k * dt, s2, n)
    var = x.var()
    assert abs(var - exact) < 4 * exact * np.sqrt(2.0 / n_paths), (var, exact)
    assert abs(x.mean()) < 4 * np.sqrt(exact / n_paths)
    return var / exact


@pytest.mark.parametrize("pot", [P1, P2])
@pytest.mark.parametrize("gamma", [0.4, 2.5])
def test_overdamped_boltzmann(orc, pot, gamma):
    check_boltzmann(orc, pot, gamma)


@pytest.mark.parametrize("scheme", [HEUN, EULER])
@pytest.mark.parametrize("pot", [P1, P2])
@pytest.mark.parametrize("gamma", [0.4, 2.5])
def test_overdamped_relaxation(orc, pot, gamma, scheme):
    check_relaxation(orc, pot, gamma, scheme)


def test_relaxation_formula_limits():
    """The discrete OU variance tends to 2 D t/gamma at short times and to
    the continuum D/V'' at long ones (the closed form itself, no oracle)."""
    D, gamma, curv, dt = 0.3, 2.0, 1.0, 1e-4
    s2, h = 2 * D * dt / gamma, curv * dt / gamma
    assert _ou_var(HEUN, h, s2, 10) == pytest.approx(2 * D * 10 * dt / gamma, rel=1e-3)
    assert _ou_var(HEUN, h, s2, 10 ** 7) == pytest.approx(D / curv, rel=1e-6)
    assert _ou_var(EULER, h, s2, 10 ** 7) == pytest.approx(D / curv, rel=1e-4)


ORACLE_C = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "oracle.c")

# (text in oracle.c, its wrong replacement)
MUTANTS = {
    "noise_without_1/gamma": (": sqrt(2.0 * P->D * dt / P->gamma);", ": sqrt(2.0 * P->D * dt);"),
    "noise_times_gamma": (": sqrt(2.0 * P->D * dt / P->gamma);", ": sqrt(2.0 * P->D * dt * P->gamma);"),
    "noise_1/gamma^2": (": sqrt(2.0 * P->D * dt / P->gamma);", ": sqrt(2.0 * P->D * dt) / P->gamma;"),
    "drift_without_1/gamma": ("F[0] = force / P->gamma;", "F[0] = force;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_a_wrong_overdamped_oracle(orc, tmp_path, monkeypatch, name):
    import oracle
    from oracle import build as obuild
    good, bad = MUTANTS[name]
    src = open(ORACLE_C).read()
    assert src.count(good) == 1, f"{good!r} not found once in oracle.c"
    path = tmp_path / "oracle_mutant.c"
    path.write_text(src.replace(good, bad))
    lib = obuild.build(src=str(path), out=str(tmp_path / "liboracle_mutant.so"))
    monkeypatch.setattr(oracle, "_lib", oracle.load(lib))
    failures = 0
    for check in (lambda: check_boltzmann(oracle, P1, 2.5), lambda: check_boltzmann(oracle, P1, 0.4),
                  lambda: check_relaxation(oracle, P2, 2.5, HEUN), lambda: check_relaxation(oracle, P1, 0.4, EULER)):
        try:
            check()
        except AssertionError:
            failures += 1
    assert failures >= 2, f"the mutant {name} passed {4 - failures} of 4 pins"
