"""The ensemble density over time of Fig. 2 (left panel; Sec. 5): windings of
every path streamed every `record_every` steps during integration
(sde_jj_integrate_recorded) and counted per row (sde_position_histograms).

Checks:
  * recording does not change the trajectory: final state bit-identical to
    sde_jj_integrate, and row r equal bit for bit to the final winding of a
    plain call that stops at that step;
  * rows against the oracle run in segments of record_every steps (its
    resume is bit-identical to one run): where per-path agreement holds
    (400 steps per period, <= 100 steps, relative error <= 1e-5 on x), the
    recorded winding equals floor(x_oracle) except where x_oracle lies within
    1e-4 of an integer (either side of the boundary is then correct);
  * the Fig. 2 density at 10 times, GPU against oracle ensembles: two-sample
    chi-square per row, p > 1e-4;
  * batched histograms bit-exact against numpy (integer work), including
    more rows than one grid dimension holds and the global-atomics path.
"""
import ctypes

import numpy as np
import pytest
import torch
from scipy import stats

import oracle
import sde_inputs

pytestmark = pytest.mark.gpu
P2 = sde_inputs.POT_SIN2PI


def _state(n, dev):
    return (torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty(n, dtype=torch.float32, device=dev), torch.empty(n, dtype=torch.float64, device=dev))


def _rows_needed(pt, step0, every):
    return (step0 + pt["n_steps"]) // every - step0 // every


def _hist_np(w, x0, nb):
    w = np.asarray(w, dtype=np.int64)
    out = np.zeros(nb + 2, dtype=np.int64)
    out[0] = np.count_nonzero(w < x0)
    out[nb + 1] = np.count_nonzero(w >= x0 + nb)
    inside = w[(w >= x0) & (w < x0 + nb)] - x0
    out[1:nb + 1] = np.bincount(inside, minlength=nb)
    return out


def test_recording_keeps_the_trajectory_and_rows_match_plain_calls(gpu):
    """Mixed kinds and lengths in one call, a nonzero step0: the final state
    equals sde_jj_integrate's, each row equals a plain call stopped at its
    step, rows past a point's last step keep their contents."""
    sde, ctx, dev = gpu
    pts = [sde_inputs.jj_point(m=m, gamma=1.1, f=f, D=0.01, n_paths=np_, steps_per_period=200, n_steps=ns,
                               potential=pot)
           for m, f, np_, ns, pot in [(1.0, 0.2, 300, 404, 0), (0.0, 1.2, 70, 196, 0), (1.0, 0.1, 129, 300, 1),
                                      (0.0, 7.0, 64, 64, 1)]]
    every, step0, seed = 32, 4, 31
    n = sum(p["n_paths"] for p in pts)
    rows = max(_rows_needed(p, step0, every) for p in pts)
    rec = torch.full((rows, n), -777, dtype=torch.int32, device=dev)
    a = _state(n, dev)
    sde.sde_jj_integrate_recorded(ctx, pts, sde.make_run(seed, step0=step0, sync=1), every, rec, *a)
    b = _state(n, dev)
    sde.sde_jj_integrate(ctx, pts, sde.make_run(seed, step0=step0, sync=1), *b)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    got = rec.cpu().numpy()
    firsts = [0]
    for p in pts:
        firsts.append(firsts[-1] + p["n_paths"])
    for r in range(rows):
        stop = (step0 // every + r + 1) * every  # absolute step of row r
        cut = [dict(p, n_steps=max(0, min(p["n_steps"], stop - step0))) for p in pts]
        c = _state(n, dev)
        sde.sde_jj_integrate(ctx, cut, sde.make_run(seed, step0=step0, sync=1), *c)
        cw = c[1].cpu().numpy()
        for q, p in enumerate(pts):
            sl = slice(firsts[q], firsts[q + 1])
            if r < _rows_needed(p, step0, every):
                assert np.array_equal(got[r, sl], cw[sl]), (r, q)
            else:
                assert (got[r, sl] == -777).all(), (r, q)


@pytest.mark.parametrize("pot", [0, P2])
@pytest.mark.parametrize("step0", [0, 4])
def test_recorded_windings_vs_oracle(gpu, pot, step0):
    """400 steps per period, 96 steps recorded every 8: every row against the
    oracle's floor(x) at the same step."""
    sde, ctx, dev = gpu
    pt = sde_inputs.jj_point(n_paths=2048, steps_per_period=400, n_steps=96, potential=pot)
    seed, every = sde_inputs.seed_of(21), 8
    n = pt["n_paths"]
    rows = _rows_needed(pt, step0, every)
    rec = torch.zeros((rows, n), dtype=torch.int32, device=dev)
    st = _state(n, dev)
    # step0 > 0 starts from the oracle's state at step0 (shared initial state)
    period = 2 * np.pi if pot == 0 else 1.0
    if step0:
        ref0 = oracle.jj_integrate([dict(pt, n_steps=step0)], seed)
        x = ref0["phi"] / period
        w = np.floor(x)
        th = (x - w).astype(np.float32)
        wrap = th >= 1.0
        th[wrap] = 0.0
        w[wrap] += 1
        st = (torch.from_numpy(th).to(dev), torch.from_numpy(w.astype(np.int32)).to(dev),
              torch.from_numpy(ref0["v"].astype(np.float32)).to(dev), torch.zeros(n, dtype=torch.float64, device=dev))
        state = (ref0["phi"], ref0["v"], ref0["acc"])
        init = sde.SDE_INIT_FROM_STATE
    else:
        state, init = None, sde.SDE_INIT_PHILOX
    sde.sde_jj_integrate_recorded(ctx, [pt], sde.make_run(seed, step0=step0, init=init, sync=1), every, rec, *st)
    got = rec.cpu().numpy()
    s = step0
    bad = 0
    for r in range(rows):
        stop = (step0 // every + r + 1) * every
        ref = oracle.jj_integrate([dict(pt, n_steps=stop - s)], seed, step0=s, state=state)
        state, s = (ref["phi"], ref["v"], ref["acc"]), stop
        x = ref["phi"] / period
        near = np.abs(x - np.round(x)) <= 1e-4 * np.maximum(1.0, np.abs(x))
        mism = got[r] != np.floor(x)
        assert not (mism & ~near).any(), (r, np.flatnonzero(mism & ~near)[:5])
        bad += int(mism.sum())
    print(f"potential {pot}, step0 {step0}: {rows} rows, {bad} windings on an integer boundary")


def test_fig2_density_vs_oracle(gpu):
    """Fig. 2 point, 2^14 paths, 100 drive periods recorded every 10 periods:
    each of the 10 rows' 200-bin histograms against the oracle ensemble."""
    sde, ctx, dev = gpu
    pt = dict(sde_inputs.jj_fig2(n_paths=1 << 14)[0], n_steps=10000)
    seed, every = sde_inputs.seed_of(22), 1000
    n = pt["n_paths"]
    rec = torch.zeros((10, n), dtype=torch.int32, device=dev)
    sde.sde_jj_integrate_recorded(ctx, [pt], sde.make_run(seed, sync=1), every, rec, *_state(n, dev))
    state = None
    worst = 1.0
    for r in range(10):
        ref = oracle.jj_integrate([dict(pt, n_steps=every)], seed, step0=r * every, state=state)
        state = (ref["phi"], ref["v"], ref["acc"])
        w_orc = np.floor(ref["phi"]).astype(np.int64)
        x0 = int(np.median(w_orc)) - 100
        counts = torch.zeros((1, 202), dtype=torch.int64, device=dev)
        sde.sde_position_histograms(ctx, rec[r:r + 1], x0, 200, counts)
        torch.cuda.synchronize()
        h_gpu = counts.cpu().numpy()[0]
        assert np.array_equal(h_gpu, _hist_np(rec[r].cpu().numpy(), x0, 200))
        h_orc = _hist_np(w_orc, x0, 200)
        keep = (h_gpu + h_orc) >= 10
        a, b = h_gpu[keep], h_orc[keep]
        chi2 = float((((a - b) ** 2) / (a + b)).sum())
        p = stats.chi2.sf(chi2, max(int(keep.sum()) - 1, 1))
        worst = min(worst, p)
        assert p > 1e-4, (r, chi2, keep.sum())
    print(f"Fig. 2 density over 10 times: smallest chi-square p = {worst:.3g}")


@pytest.mark.parametrize("rows,n,pitch,nb", [(1, 1000, 1000, 200), (7, 1001, 1024, 200), (3, 5000, 5000, 9000),
                                             (70000, 3, 4, 5), (2, 0, 8, 10)])
def test_batched_histograms_bit_exact(gpu, rows, n, pitch, nb):
    sde, ctx, dev = gpu
    rng = np.random.default_rng(rows + n + nb)
    x0 = -nb // 3
    w = rng.integers(x0 - nb // 2 - 2, x0 + nb + nb // 2 + 2, (rows, pitch)).astype(np.int32)
    wt = torch.from_numpy(w).to(dev)
    counts = torch.full((rows, nb + 2), 999, dtype=torch.int64, device=dev)
    sde.sde_position_histograms(ctx, wt, x0, nb, counts, n=n)
    torch.cuda.synchronize()
    got = counts.cpu().numpy()
    for r in range(rows) if rows < 100 else list(range(50)) + list(range(rows - 50, rows)):
        assert np.array_equal(got[r], _hist_np(w[r, :n], x0, nb)), r
    assert (got.sum(axis=1) == n).all()


def test_recorded_invalid_arguments_leave_outputs(gpu):
    sde, ctx, dev = gpu
    pt = sde_inputs.jj_point(n_paths=64, n_steps=40)
    st = _state(64, dev)
    for x in st:
        x.zero_()
    rec = torch.zeros((5, 64), dtype=torch.int32, device=dev)
    for every, r in [(6, rec), (0, rec), (8, rec[:4]), (8, None)]:
        with pytest.raises(sde.SDEError) as e:
            sde.sde_jj_integrate_recorded(ctx, [pt], sde.make_run(1, sync=1), every, r, *st)
        assert e.value.status == sde.SDE_ERR_INVALID
    # misaligned record buffer (raw pointer 2 bytes into the tensor)
    L = sde.lib()
    pts = sde.make_points([pt])
    run = sde.make_run(1, sync=1)
    rc = L.sde_jj_integrate_recorded(ctx, pts, 1, ctypes.byref(run), st[0].data_ptr(), st[1].data_ptr(),
                                     st[2].data_ptr(), st[3].data_ptr(), None, 8, 5, rec.data_ptr() + 2, None)
    assert rc == sde.SDE_ERR_INVALID
    assert all(torch.count_nonzero(x) == 0 for x in st)
    assert torch.count_nonzero(rec) == 0
    # exactly enough rows is accepted
    sde.sde_jj_integrate_recorded(ctx, [pt], sde.make_run(1, sync=1), 8, rec, *st)
    assert torch.count_nonzero(rec) >= 0
    counts = torch.zeros((2, 12), dtype=torch.int64, device=dev)
    w = torch.zeros((2, 8), dtype=torch.int32, device=dev)
    with pytest.raises(sde.SDEError):
        sde.sde_position_histograms(ctx, w, 0, 10, counts, n=9)  # pitch < n with several rows


def test_recorded_graph_follows_the_path_count(gpu):
    """Graphs on (the default), the same buffers, 2 paths per lane (one
    128-path chunk): recorded calls at 128, 100 and again 128 paths.  The
    row pitch is the call's path count, so the 100-path call must not replay
    the 128-path graph; each call equals the same call with graphs off, the
    record buffer of the 100-path call is exactly rows x 100, and what lies
    beyond it in the storage keeps its contents.  The third call replays the
    first one's graph."""
    sde, ctx, dev = gpu
    sde.sde_set_option(ctx, sde.SDE_OPT_JJ_PPT, 2)
    every, seed, n_steps = 8, 41, 64
    rows = n_steps // every
    store = torch.full((rows * 128 + 512,), -5, dtype=torch.int32, device=dev)
    st = _state(128, dev)
    replayed = []
    for n in (128, 100, 128):
        pt = [sde_inputs.jj_point(n_paths=n, n_steps=n_steps, D=0.01, steps_per_period=200)]
        assert _rows_needed(pt[0], 0, every) == rows
        store.fill_(-5)
        rec = store[:rows * n].view(rows, n)
        sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, 1)
        sde.sde_jj_integrate_recorded(ctx, pt, sde.make_run(seed, sync=1), every, rec, *(x[:n] for x in st))
        replayed.append(sde.sde_get_stats(ctx)["graph_replayed"])
        sde.sde_set_option(ctx, sde.SDE_OPT_GRAPHS, 0)
        rec_e = torch.full((rows, n), -5, dtype=torch.int32, device=dev)
        st_e = _state(n, dev)
        sde.sde_jj_integrate_recorded(ctx, pt, sde.make_run(seed, sync=1), every, rec_e, *st_e)
        assert torch.equal(rec, rec_e), n
        for x, y in zip(st, st_e):
            assert torch.equal(x[:n], y), n
        assert bool((store[rows * n:] == -5).all()), n
    assert replayed[2] == 1, replayed
