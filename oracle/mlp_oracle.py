"""FP64 NumPy reference of the learned amplitude start (test infrastructure).

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and bench.py's
cpu_baseline leg may import or call this; the product never does.

The learned start maps per-element features of the first-order amplitudes to
a correction of them (the paper has no network of its own; its only mentions
of machine learning concern dispatch, Sec. 3.2 and Sec. 5). Reading used here:
  * features of element (i, j, a, b):
        x = (t_MP2 / sigma, D_ij^ab, e_i + e_j, e_a + e_b),
    sigma = RMS of t_MP2 over the instance; every feature is invariant under
    (i,j,a,b) -> (j,i,b,a), so the guess keeps the amplitudes' pair symmetry;
  * network 4 -> H -> H -> 1 with SiLU after the two hidden layers;
  * target (t* - t_MP2) / sigma, mean squared error;
  * guess t = t_MP2 + sigma * f(x);
  * Adam with bias correction.
Parameters are a dict of arrays: W1 [H,4], b1 [H], W2 [H,H], b2 [H], W3 [H], b3 [1].
"""
from __future__ import annotations

import numpy as np

__all__ = ["silu", "dsilu", "init_params", "forward", "loss", "grad", "adam_step",
           "features", "targets", "flatten", "unflatten", "PARAM_ORDER"]

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def init_params(width=128, seed=0):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases (a plain choice)."""
    rng = np.random.default_rng(seed)
    H = width

    def u(shape, fan_in):
        b = 1.0 / np.sqrt(fan_in)
        return rng.uniform(-b, b, size=shape)
    return {"W1": u((H, 4), 4), "b1": u((H,), 4), "W2": u((H, H), H), "b2": u((H,), H),
            "W3": u((H,), H), "b3": u((1,), H)}


def forward(p, X):
    """Returns (y, cache) for X [n, 4]."""
    Z1 = X @ p["W1"].T + p["b1"]
    H1 = silu(Z1)
    Z2 = H1 @ p["W2"].T + p["b2"]
    H2 = silu(Z2)
    y = H2 @ p["W3"] + p["b3"][0]
    return y, (X, Z1, H1, Z2, H2)


def loss(p, X, Y):
    y, _ = forward(p, X)
    return float(np.mean((y - Y) ** 2))


def grad(p, X, Y):
    """Gradient of the mean squared error with respect to every parameter (backpropagation)."""
    y, (X, Z1, H1, Z2, H2) = forward(p, X)
    n = X.shape[0]
    dy = 2.0 * (y - Y) / n                 # [n]
    g = {}
    g["W3"] = H2.T @ dy                    # [H]
    g["b3"] = np.array([dy.sum()])
    dZ2 = np.outer(dy, p["W3"]) * dsilu(Z2)  # [n, H]
    g["W2"] = dZ2.T @ H1                   # [H, H]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ p["W2"]) * dsilu(Z1)      # [n, H]
    g["W1"] = dZ1.T @ X                    # [H, 4]
    g["b1"] = dZ1.sum(axis=0)
    return g


def adam_step(p, g, state, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in place; state = {'t': int, 'm': dict, 'v': dict}."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    m = state.setdefault("m", {k: np.zeros_like(v) for k, v in p.items()})
    v = state.setdefault("v", {k: np.zeros_like(v) for k, v in p.items()})
    for k in p:
        m[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1.0 - beta2) * g[k] ** 2
        mh = m[k] / (1.0 - beta1 ** t)
        vh = v[k] / (1.0 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def features(t_mp2, e_occ, e_vir):
    """X [o*o*v*v, 4] in (i, j, a, b) order and sigma = RMS(t_MP2)."""
    o, _, v, _ = t_mp2.shape
    sigma = float(np.sqrt(np.mean(t_mp2 ** 2)))
    eij = (e_occ[:, None] + e_occ[None, :])[:, :, None, None] * np.ones((1, 1, v, v))
    eab = (e_vir[:, None] + e_vir[None, :])[None, None, :, :] * np.ones((o, o, 1, 1))
    D = eij - eab
    X = np.stack([t_mp2 / sigma, D, eij, eab], axis=-1).reshape(-1, 4)
    return X, sigma


def targets(t_star, t_mp2, sigma):
    return ((t_star - t_mp2) / sigma).reshape(-1)


def flatten(p):
    """Parameters in the library's flat order: W1 (row-major), b1, W2, b2, W3, b3."""
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in PARAM_ORDER])


def unflatten(flat, width=128):
    H = width
    sizes = {"W1": (H, 4), "b1": (H,), "W2": (H, H), "b2": (H,), "W3": (H,), "b3": (1,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(sizes[k]))
        out[k] = np.array(flat[o:o + n], dtype=np.float64).reshape(sizes[k])
        o += n
    return out
