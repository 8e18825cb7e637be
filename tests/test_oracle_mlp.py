"""Pins of the oracle MLP (CPU only): torch's reference layers and autograd
in float64, central finite differences, the closed-form first Adam step and
torch.optim.Adam."""
import numpy as np
import torch

import oracle.mlp as om

WIDTHS = [5, 16, 12, 9, 1]


def _params(seed=0, widths=WIDTHS):
    rng = np.random.default_rng(seed)
    ps = []
    for (o, i), _ in om.param_shapes(widths):
        bound = 1.0 / np.sqrt(i)
        ps.append((rng.uniform(-bound, bound, (o, i)), rng.uniform(-bound, bound, o)))
    return ps


def _torch_forward(params, X):
    h = torch.from_numpy(X)
    for l, (W, b) in enumerate(params):
        h = torch.nn.functional.linear(h, torch.from_numpy(W), torch.from_numpy(b))
        if l < len(params) - 1:
            h = torch.nn.functional.gelu(h, approximate="none")
    return h[:, 0]


def test_forward_matches_torch():
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (33, 5))
    ps = _params()
    y, _, _ = om.forward(ps, X)
    np.testing.assert_allclose(y, _torch_forward(ps, X).numpy(), rtol=1e-13, atol=1e-14)


def test_gelu_and_derivative():
    z = np.linspace(-6, 6, 1001)
    np.testing.assert_allclose(om.gelu(z), torch.nn.functional.gelu(torch.from_numpy(z)).numpy(),
                               rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def test_gradients_match_autograd():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (40, 5))
    t = rng.standard_normal(40)
    ps = _params(3)
    loss, grads = om.loss_and_grad(ps, X, t)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in ps]
    h = torch.from_numpy(X)
    for l, (W, b) in enumerate(tp):
        h = torch.nn.functional.linear(h, W, b)
        if l < len(tp) - 1:
            h = torch.nn.functional.gelu(h, approximate="none")
    tl = torch.mean((h[:, 0] - torch.from_numpy(t)) ** 2)
    tl.backward()
    assert abs(loss - tl.item()) < 1e-14
    for (gW, gb), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(gW, W.grad.numpy(), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (20, 5))
    t = rng.standard_normal(20)
    ps = _params(5)
    _, grads = om.loss_and_grad(ps, X, t)
    flat = om.pack(ps)
    g = om.pack(grads)
    h = 1e-6
    idx = rng.choice(flat.size, 60, replace=False)
    for k in idx:
        fp, fm = flat.copy(), flat.copy()
        fp[k] += h
        fm[k] -= h
        lp, _ = om.loss_and_grad(om.unpack(fp, WIDTHS), X, t)
        lm, _ = om.loss_and_grad(om.unpack(fm, WIDTHS), X, t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-3), (k, fd, g[k])


def test_pack_roundtrip_and_count():
    ps = _params(6)
    flat = om.pack(ps)
    assert flat.size == om.n_params(WIDTHS)
    assert om.n_params([5, 256, 256, 256, 1]) == 133377
    for (W, b), (W2, b2) in zip(ps, om.unpack(flat, WIDTHS)):
        assert np.array_equal(W, W2) and np.array_equal(b, b2)


def test_first_adam_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (25, 5))
    t = rng.standard_normal(25)
    ps = _params(8)
    _, grads = om.loss_and_grad(ps, X, t)
    new = om.adam_step(ps, grads, om.zeros_like(ps), om.zeros_like(ps), 1, lr=1e-3)
    for (W, b), (gW, gb), (W1, b1) in zip(ps, grads, new):
        np.testing.assert_allclose(W1 - W, -1e-3 * gW / (np.abs(gW) + 1e-8), rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(b1 - b, -1e-3 * gb / (np.abs(gb) + 1e-8), rtol=1e-9, atol=1e-15)


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(9)
    X = rng.uniform(-1, 1, (30, 5))
    t = rng.standard_normal(30)
    ps = _params(10)
    tp = [torch.tensor(a, requires_grad=True) for W, b in ps for a in (W, b)]
    opt = torch.optim.Adam(tp, lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m, v = om.zeros_like(ps), om.zeros_like(ps)
    cur = ps
    for step in range(1, 6):
        _, grads = om.loss_and_grad(cur, X, t)
        cur = om.adam_step(cur, grads, m, v, step)
        opt.zero_grad()
        h = torch.from_numpy(X)
        for l in range(len(ps)):
            h = torch.nn.functional.linear(h, tp[2 * l], tp[2 * l + 1])
            if l < len(ps) - 1:
                h = torch.nn.functional.gelu(h, approximate="none")
        torch.mean((h[:, 0] - torch.from_numpy(t)) ** 2).backward()
        opt.step()
    for l, (W, b) in enumerate(cur):
        np.testing.assert_allclose(W, tp[2 * l].detach().numpy(), rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(b, tp[2 * l + 1].detach().numpy(), rtol=1e-10, atol=1e-13)
