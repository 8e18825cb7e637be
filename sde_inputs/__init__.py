"""Seeded synthetic inputs for the five workloads (no method arithmetic).

This module is the only code shared by the HIP library's callers and the CPU
oracle: it builds parameter sets, natural frequencies and coupling matrices
from numpy's seeded generator.  It computes no step of the method itself;
the random numbers the method draws while integrating (initial conditions,
per-step noise) come from each side's own Philox4x32-10.

Workloads (all parameters from the paper's models, Eq. 1 and Eq. 2):
  jj_single   one Josephson-junction point with the parameters of the
              paper's Fig. 2 run (a=4.2, gamma=0.9, omega=4.9, D=0.001,
              f=0.1), 4096 paths, dt = 2 pi / omega / 400, 10^4 steps
  jj_scan     128 x 128 (f, D) grid: f = 0.5 i/127, D = 10^(-4 + 3 j/127),
              point index q = 128 i + j; 1024 paths, 2*10^5 steps of
              dt = 2 pi / omega / 200, the first 10^5 discarded
  kuramoto_uniform  N = 65536, omega_i ~ N(0, 1), K = 3, D = 0.1, dt = 0.01,
              16 realizations
  kuramoto_dense    N = 4096, K_ij = (K/N)(1 + 0.5 u_ij), u_ij ~ U[-1, 1]
              symmetric, zero diagonal, K = 4, omega_i ~ N(0, 0.5), D = 0.05,
              dt = 0.005, 256 realizations
  jj_batch    2048 random points: a ~ U[2,6], omega ~ U[3,7], f ~ U[0,0.5],
              log10 D ~ U[-4,-1], gamma ~ U[0.5,1.5], m = 1; paths uniform
              in {256..8192}, steps uniform in {5*10^4..4*10^5}, transient
              floor(steps/2), dt = 2 pi / omega / 200
"""
import numpy as np

SEED_BASE = 9033852


def seed_of(k):
    """Seed of workload k (1 = jj_single ... 5 = jj_batch)."""
    return SEED_BASE + k


POT_SIN, POT_SIN2PI = 0, 1  # -sin(phi) force (Josephson form); V(x) = sin(2 pi x)


def jj_point(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=0.1, D=1e-3, n_paths=4096,
             steps_per_period=400, n_steps=10000, n_transient=0, potential=POT_SIN):
    return dict(m=float(m), gamma=float(gamma), a=float(a), omega=float(omega), f=float(f),
                D=float(D), n_paths=int(n_paths), steps_per_period=int(steps_per_period),
                n_steps=int(n_steps), n_transient=int(n_transient), potential=int(potential))


def jj_fig2(n_paths=1 << 19, periods=2000):
    """The ensemble of the paper's precision study (Fig. 2): V(x) = sin(2 pi x),
    a = 4.2, gamma = 0.9, omega = 4.9, D = 0.001, f = 0.1, dt = 0.01 of the
    drive period, t in (0, 2000 periods); the position histogram at the end
    has 200 bins of one potential period."""
    return [jj_point(m=1.0, gamma=0.9, a=4.2, omega=4.9, f=0.1, D=1e-3, n_paths=n_paths,
                     steps_per_period=100, n_steps=100 * periods, n_transient=0,
                     potential=POT_SIN2PI)]


def jj_single(n_paths=4096, n_steps=10000):
    return [jj_point(n_paths=n_paths, n_steps=n_steps)]


def jj_scan_fd(i, j):
    return 0.5 * i / 127.0, 10.0 ** (-4.0 + 3.0 * j / 127.0)


def jj_scan(n_paths=1024, n_steps=200000, n_transient=100000, indices=None):
    """Points of the (f, D) scan.  `indices` = iterable of q = 128 i + j
    (default: all 16384 in order)."""
    qs = range(128 * 128) if indices is None else indices
    pts = []
    for q in qs:
        f, D = jj_scan_fd(q // 128, q % 128)
        pts.append(jj_point(f=f, D=D, n_paths=n_paths, steps_per_period=200,
                            n_steps=n_steps, n_transient=n_transient))
    return pts


def kuramoto_omega(N, sigma, seed):
    """Natural frequencies, float32 (the device dtype); the oracle receives
    the same values widened to float64."""
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal(N)).astype(np.float32)


def kuramoto_uniform(N=65536, R=16):
    return dict(N=N, R=R, K=3.0, D=0.1, dt=0.01, n_steps=100000, sample_every=100,
                omega=kuramoto_omega(N, 1.0, seed_of(3)), seed=seed_of(3))


def kuramoto_fig4(N=1 << 24, n_steps=2000):
    """The globally coupled system of Fig. 4: 2^24 identical oscillators
    (omega_i = 0), K = 4, T = 1 (D = 1), one realization, uniform random
    initial phases, dt = 0.01; r(t) and the phase density every 100 steps."""
    return dict(N=N, R=1, K=4.0, D=1.0, dt=0.01, n_steps=n_steps, sample_every=100,
                omega=np.zeros(N, dtype=np.float32), seed=seed_of(6))


def dense_coupling(N, K, seed):
    """Symmetric K_ij = (K/N)(1 + 0.5 u_ij), u_ij ~ U[-1,1], zero diagonal, float32."""
    rng = np.random.default_rng(seed + 1)
    u = rng.uniform(-1.0, 1.0, size=(N, N))
    u = np.triu(u, 1)
    u = u + u.T
    Kmat = (K / N) * (1.0 + 0.5 * u)
    np.fill_diagonal(Kmat, 0.0)
    return Kmat.astype(np.float32)


def kuramoto_dense(N=4096, R=256):
    return dict(N=N, R=R, K=4.0, D=0.05, dt=0.005, n_steps=20000, sample_every=100,
                omega=kuramoto_omega(N, 0.5, seed_of(4)), Kmat=dense_coupling(N, 4.0, seed_of(4)),
                seed=seed_of(4))


def jj_anm_params(n, seed):
    """(a, omega, f, D, gamma) rows around the paper's Fig. 2 point in its own
    potential V(x) = sin(2 pi x), where the mean velocity changes sign and
    magnitude (anomalous response): a ~ U[3.5, 5], omega ~ U[4, 6],
    f ~ U[-0.3, 0.3], log10 D ~ U[-4, -2], gamma ~ U[0.7, 1.2]."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(3.5, 5.0, n)
    om = rng.uniform(4.0, 6.0, n)
    f = rng.uniform(-0.3, 0.3, n)
    D = 10.0 ** rng.uniform(-4.0, -2.0, n)
    g = rng.uniform(0.7, 1.2, n)
    return np.stack([a, om, f, D, g], axis=1)


def jj_random_params(n, seed):
    """(a, omega, f, D, gamma) rows drawn from the batch distribution."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(2.0, 6.0, n)
    om = rng.uniform(3.0, 7.0, n)
    f = rng.uniform(0.0, 0.5, n)
    D = 10.0 ** rng.uniform(-4.0, -1.0, n)
    g = rng.uniform(0.5, 1.5, n)
    return np.stack([a, om, f, D, g], axis=1)


def jj_batch(n_points=2048, seed=None, path_range=(256, 8192), step_range=(50000, 400000)):
    seed = seed_of(5) if seed is None else seed
    P = jj_random_params(n_points, seed)
    rng = np.random.default_rng(seed + 7)
    paths = rng.integers(path_range[0], path_range[1] + 1, n_points)
    steps = rng.integers(step_range[0], step_range[1] + 1, n_points)
    return [jj_point(a=p[0], omega=p[1], f=p[2], D=p[3], gamma=p[4], n_paths=int(npth),
                     steps_per_period=200, n_steps=int(ns), n_transient=int(ns) // 2)
            for p, npth, ns in zip(P, paths, steps)]
