"""The per-pair MLP of the learned coarse correction and its training loss (float64).

Test infrastructure only (see ``oracle/__init__.py``).

Network: features (8) -> tanh(64) -> tanh(64) -> linear(278) = (theta_off, theta_self),
weights flattened as W1 (8 x 64, row-major, in x out), b1 (64), W2 (64 x 64), b2 (64),
W3 (64 x 278), b3 (278).

Loss over a training set of configurations, each with directed near pairs, their
features and directions, and n_rhs samples (xi = low-mode coefficients of a right-hand
side, t = R x - R M0 b for the solution x of A x = b with b = P xi):
    L = sum |t - zeta(xi)|^2 / sum |t|^2,   zeta from oracle.coarse.coarse_apply.

Parity: gradients pinned by central finite differences (tests/test_oracle_coarse.py).
"""
import numpy as np

from .coarse import NFEAT, NTHETA, K_from_theta, pair_frame, rot25, theta_grad_from_K

HIDDEN = 64
NOUT = 2 * NTHETA


def layer_shapes():
    return [(NFEAT, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, NOUT), (NOUT,)]


def n_weights():
    return sum(int(np.prod(s)) for s in layer_shapes())


def unpack(wflat):
    out, o = [], 0
    for s in layer_shapes():
        n = int(np.prod(s))
        out.append(np.asarray(wflat[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def forward(wflat, X):
    W1, b1, W2, b2, W3, b3 = unpack(wflat)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    y = h2 @ W3 + b3
    return y, (X, h1, h2)


def backward(wflat, cache, dy):
    W1, b1, W2, b2, W3, b3 = unpack(wflat)
    X, h1, h2 = cache
    dW3 = h2.T @ dy
    db3 = dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (1.0 - h2 * h2)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (1.0 - h1 * h1)
    dW1 = X.T @ dh1
    db1 = dh1.sum(axis=0)
    return np.concatenate([a.reshape(-1) for a in (dW1, db1, dW2, db2, dW3, db3)])


def predict(pairs, dirs, theta, xi):
    """zeta for every sample: xi (R, nb, 25) -> (R, nb, 25)."""
    out = np.zeros_like(xi)
    for e, (i, j) in enumerate(pairs):
        Rm = rot25(pair_frame(dirs[e]))
        Ko = K_from_theta(theta[e, :NTHETA])
        Ks = K_from_theta(theta[e, NTHETA:])
        out[:, i] += (Rm.T @ (Ko @ (Rm @ xi[:, j].T) + Ks @ (Rm @ xi[:, i].T))).T
    return out


def loss_and_grad(wflat, dataset):
    """dataset: list of dicts with pairs, feats, dirs, xi (R, nb, 25), t (R, nb, 25)."""
    den = sum(float(np.sum(d["t"] ** 2)) for d in dataset)
    num = 0.0
    grad = np.zeros(n_weights())
    for d in dataset:
        theta, cache = forward(wflat, d["feats"])
        res = d["t"] - predict(d["pairs"], d["dirs"], theta, d["xi"])
        num += float(np.sum(res ** 2))
        gpred = -2.0 * res / den
        dtheta = np.zeros_like(theta)
        for e, (i, j) in enumerate(d["pairs"]):
            Rm = rot25(pair_frame(d["dirs"][e]))
            u = Rm @ gpred[:, i].T                 # (25, R)
            dKo = u @ (Rm @ d["xi"][:, j].T).T
            dKs = u @ (Rm @ d["xi"][:, i].T).T
            dtheta[e, :NTHETA] = theta_grad_from_K(dKo)
            dtheta[e, NTHETA:] = theta_grad_from_K(dKs)
        grad += backward(wflat, cache, dtheta)
    return num / den, grad


def init_weights(seed=0, out_scale=1e-3):
    """Glorot-uniform hidden layers, small output layer (the correction starts at 0)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in layer_shapes():
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            if s[1] == NOUT:
                lim *= out_scale
            parts.append(rng.uniform(-lim, lim, s))
    return np.concatenate([p.reshape(-1) for p in parts])
