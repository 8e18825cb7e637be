"""The small-N remedy of the all-pairs (Alg. 3) sum: the j range split over
J workgroup slices whose partial sums are added in slice order (Sec. 6:
less work per thread, more threads, when N alone cannot fill the device).

Checks: against the FP64 oracle, first 100 steps under shared noise, per
oscillator |d phi| <= 1e-5 max(|phi|, 1) (the bound of the unsplit kernel)
for forced and automatic J, Heun and Euler-Maruyama, ragged slices; split
and unsplit agree to twice that bound; the automatic choice splits only
launches that leave the device idle; a split run resumes bit for bit.
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


def _tiled(gpu, N, R, n_steps, J, scheme=0, seed=3, phi=None, step0=0):
    sde, ctx, dev = gpu
    cfg = sde_inputs.kuramoto_uniform(N=N, R=R)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_JSPLIT, J)
    om = torch.from_numpy(cfg["omega"]).to(dev)
    ph = phi if phi is not None else torch.empty((R, N), dtype=torch.float32, device=dev)
    init = sde.SDE_INIT_FROM_STATE if phi is not None else sde.SDE_INIT_PHILOX
    rs = torch.zeros((R, n_steps // 100 + 1), dtype=torch.float64, device=dev)
    desc = sde.sde_kuramoto_desc(N, R, cfg["K"], cfg["D"], cfg["dt"], n_steps, sde.SDE_TILED, 0)
    sde.sde_kuramoto_integrate(ctx, desc, sde.make_run(seed, step0=step0, scheme=scheme, init=init, sync=1), ph, om,
                               None, rs)
    return ph, rs, sde.sde_get_stats(ctx)["kura_jsplit"], cfg


@pytest.mark.parametrize("N,R,J", [(4096, 1, 1), (4096, 1, 7), (4096, 1, 64), (1000, 3, 0), (5000, 2, 0),
                                   (4096, 1, 0)])
@pytest.mark.parametrize("scheme", [0, 1])
def test_split_sum_vs_oracle(gpu, N, R, J, scheme):
    ph, rs, used, cfg = _tiled(gpu, N, R, 100, J, scheme)
    if J:
        assert used == J
    else:
        assert used > 1  # these launches alone would leave the device idle
    ref, rref = oracle.kuramoto_integrate(N, R, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD, scheme,
                                          3, cfg["omega"].astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"N {N} R {R} J {used} scheme {scheme}: max phase error {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_split_matches_unsplit(gpu):
    a, ra, ja, _ = _tiled(gpu, 8192, 1, 100, 1)
    b, rb, jb, _ = _tiled(gpu, 8192, 1, 100, 0)
    assert ja == 1 and jb > 1
    err = _circ_err(a.cpu().numpy(), 2 * np.pi * b.cpu().numpy().astype(np.float64))
    print(f"J = {jb} against J = 1: max phase difference {err.max():.2e}")
    assert err.max() <= 2e-5


def test_automatic_split_leaves_full_launches_alone(gpu):
    _, _, used, _ = _tiled(gpu, 65536, 16, 2, 0)
    assert used == 1


def test_split_resume_bit_identical(gpu):
    full, _, j, _ = _tiled(gpu, 3000, 1, 50, 0, seed=8)
    assert j > 1
    a, _, _, _ = _tiled(gpu, 3000, 1, 21, 0, seed=8)
    b, _, _, _ = _tiled(gpu, 3000, 1, 29, 0, seed=8, phi=a, step0=21)
    assert torch.equal(full, b)


def test_jsplit_option_validation(gpu):
    sde, ctx, dev = gpu
    for bad in (-1, 65536):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_KURA_JSPLIT, bad)


@pytest.mark.parametrize("tile", [1, 2, 4])
def test_forced_tile_vs_oracle(gpu, tile):
    """Every all-pairs tile (256 x OPT phases in LDS) against the oracle."""
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_TILE, tile)
    ph, rs, _, cfg = _tiled(gpu, 3000, 2, 100, 0)
    assert sde.sde_get_stats(ctx)["kura_tile"] == tile
    ref, rref = oracle.kuramoto_integrate(3000, 2, cfg["K"], cfg["D"], cfg["dt"], 100, 100, oracle.MEANFIELD, 0, 3,
                                          cfg["omega"].astype(np.float64))
    err = _circ_err(ph.cpu().numpy(), ref)
    print(f"tile {tile}: max phase error {err.max():.2e}")
    assert err.max() <= 1e-5
    np.testing.assert_allclose(rs.cpu().numpy(), rref, rtol=0, atol=1e-6)


def test_tile_autotuner_reads_only_and_caches(gpu):
    """The tuner times trial stages on copies: a tuned call equals a call
    forced to the chosen tile bit for bit, and the next call of the shape
    class takes the cached choice without tuning."""
    sde, _, dev = gpu
    ctx = sde.sde_create(0)  # its own (empty) tune cache
    try:
        _tile_autotuner_checks(sde, ctx, dev)
    finally:
        sde.sde_destroy(ctx)


def _tile_autotuner_checks(sde, ctx, dev):
    gpu = (sde, ctx, dev)
    a, ra, _, _ = _tiled(gpu, 8192, 2, 30, 0)
    st = sde.sde_get_stats(ctx)
    assert st["tuned"] == 1 and st["kura_tile"] in (1, 2, 4)
    chosen = st["kura_tile"]
    print(f"tuned tile {chosen} in {st['tune_ms']:.1f} ms")
    b, rb, _, _ = _tiled(gpu, 8192, 2, 30, 0)
    st2 = sde.sde_get_stats(ctx)
    assert st2["tuned"] == 0 and st2["kura_tile"] == chosen
    assert torch.equal(a, b) and torch.equal(ra, rb)
    sde.sde_set_option(ctx, sde.SDE_OPT_KURA_TILE, chosen)
    c, rc, _, _ = _tiled(gpu, 8192, 2, 30, 0)
    assert torch.equal(a, c) and torch.equal(ra, rc)
    for bad in (3, -1, 8):
        with pytest.raises(sde.SDEError):
            sde.sde_set_option(ctx, sde.SDE_OPT_KURA_TILE, bad)
