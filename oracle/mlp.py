"""Plain FP64 numpy reference of the ensemble-member MLP of the <v>
surrogate (test infrastructure only; see oracle/__init__.py).

Network: widths w_0 .. w_L (5-256-256-256-1 for the Josephson-junction
surrogate); hidden layers h_l = GELU(W_l h_{l-1} + b_l) with the exact
GELU(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2; the output layer is
linear.  Loss: mean squared error.  Optimizer: Adam (Kingma & Ba, 2015)
with bias correction.  Parameters of a member are a list of (W [out, in],
b [out]) pairs; the packed order is W_1, b_1, W_2, b_2, ... row-major.

Parity: pinned (tests/test_oracle_mlp.py) against torch's CPU layers and
autograd in float64, central finite differences, the closed-form first Adam
step and torch.optim.Adam.
"""
import math

import numpy as np

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)

try:
    from scipy.special import erf as _erf
except ImportError:  # pragma: no cover
    _erf = np.vectorize(math.erf)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / SQRT2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def param_shapes(widths):
    return [((widths[l + 1], widths[l]), (widths[l + 1],)) for l in range(len(widths) - 1)]


def n_params(widths):
    return sum(o * i + o for (o, i), _ in param_shapes(widths))


def pack(params):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in params])


def unpack(flat, widths):
    out, k = [], 0
    for (o, i), _ in param_shapes(widths):
        W = np.asarray(flat[k:k + o * i], dtype=np.float64).reshape(o, i)
        k += o * i
        b = np.asarray(flat[k:k + o], dtype=np.float64)
        k += o
        out.append((W, b))
    return out


def forward(params, X):
    """X [B, w_0] -> (output [B], list of pre-activations Z_l, list of
    layer inputs A_{l-1})."""
    A = np.asarray(X, dtype=np.float64)
    Zs, As = [], []
    for l, (W, b) in enumerate(params):
        As.append(A)
        Z = A @ W.T + b
        Zs.append(Z)
        A = gelu(Z) if l < len(params) - 1 else Z
    return A[:, 0], Zs, As


def loss_and_grad(params, X, t):
    """Mean squared error and its gradient with respect to every parameter
    (analytic back-propagation)."""
    y, Zs, As = forward(params, X)
    B = len(t)
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    dZ = (2.0 / B) * r[:, None]                   # d loss / d Z_L
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (dZ.T @ As[l], dZ.sum(axis=0))
        if l > 0:
            dA = dZ @ W                           # d loss / d A_{l-1}
            dZ = dA * gelu_grad(Zs[l - 1])
    return loss, grads


def adam_step(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t >= 1 is the update count after this step).  m, v
    are lists shaped like params (updated in place); returns new params."""
    new = []
    for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        out = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m[l][j] = beta1 * m[l][j] + (1.0 - beta1) * g
            v[l][j] = beta2 * v[l][j] + (1.0 - beta2) * g * g
            mh = m[l][j] / (1.0 - beta1 ** t)
            vh = v[l][j] / (1.0 - beta2 ** t)
            out.append(p - lr * mh / (np.sqrt(vh) + eps))
        new.append(tuple(out))
    return new


def zeros_like(params):
    return [[np.zeros_like(W), np.zeros_like(b)] for W, b in params]
