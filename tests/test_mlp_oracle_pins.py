"""Pins of the FP64 reference of the learned start: backpropagation against
central finite differences, closed forms of special parameter choices, the
Adam update against its first-step closed form, and feature invariances."""
import numpy as np
import pytest

from oracle import mlp_oracle as M
import ppl_synth as S
import oracle as O


def test_silu_derivative_matches_finite_differences():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (M.silu(z + h) - M.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - M.dsilu(z))) < 1e-9


@pytest.mark.parametrize("width", [8, 16])
def test_backprop_matches_central_differences(width):
    rng = np.random.default_rng(0)
    p = M.init_params(width, seed=1)
    X = rng.standard_normal((37, 4))
    Y = rng.standard_normal(37)
    g = M.grad(p, X, Y)
    h = 1e-6
    for k in M.PARAM_ORDER:
        flat = p[k].ravel()
        for idx in rng.choice(flat.size, size=min(12, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = M.loss(p, X, Y)
            flat[idx] = old - h
            lm = M.loss(p, X, Y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k].ravel()[idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_special_parameter_choices():
    H = 8
    p = M.init_params(H, seed=2)
    X = np.random.default_rng(3).standard_normal((20, 4))
    # zero output weights: the network is its output bias
    p0 = {k: v.copy() for k, v in p.items()}
    p0["W3"][:] = 0.0
    y, _ = M.forward(p0, X)
    assert np.all(y == p0["b3"][0])
    # zero hidden weights and biases: SiLU(0) = 0, so the output is b3 again
    p1 = {k: v.copy() for k, v in p.items()}
    p1["W2"][:] = 0.0
    p1["b2"][:] = 0.0
    y, _ = M.forward(p1, X)
    assert np.allclose(y, p1["b3"][0], atol=0)
    # one hidden unit path by hand
    p2 = {k: np.zeros_like(v) for k, v in p.items()}
    p2["W1"][0, 0] = 2.0
    p2["W2"][0, 0] = 3.0
    p2["W3"][0] = 5.0
    y, _ = M.forward(p2, X)
    assert np.allclose(y, 5.0 * M.silu(3.0 * M.silu(2.0 * X[:, 0])), rtol=1e-15)


def test_adam_first_step_is_sign_times_lr():
    p = M.init_params(8, seed=4)
    rng = np.random.default_rng(5)
    g = {k: rng.standard_normal(v.shape) for k, v in p.items()}
    before = {k: v.copy() for k, v in p.items()}
    M.adam_step(p, g, {}, lr=1e-3, eps=0.0)
    # with bias correction the first step is lr * g / |g|
    for k in p:
        assert np.allclose(before[k] - p[k], 1e-3 * np.sign(g[k]), rtol=1e-12, atol=0)


def test_features_are_pair_invariant():
    s = S.make_system(3, 6, 10, 0, "contractive")
    t = O.mp2_amplitudes(s["L"], 3, s["e_occ"], s["e_vir"])
    X, sigma = M.features(t, s["e_occ"], s["e_vir"])
    X = X.reshape(3, 3, 6, 6, 4)
    # V = (ia|jb) from a BLAS product is pair-symmetric to rounding only
    np.testing.assert_allclose(X, X.transpose(1, 0, 3, 2, 4), rtol=1e-13, atol=1e-15)
    assert abs(np.sqrt(np.mean((X[..., 0] * sigma) ** 2)) - sigma) < 1e-15
    V, D = O.mp2_parts(s["L"], 3, s["e_occ"], s["e_vir"])
    np.testing.assert_allclose(X[..., 1], D, rtol=1e-15, atol=1e-14)


def test_flatten_roundtrip():
    p = M.init_params(16, seed=6)
    q = M.unflatten(M.flatten(p), 16)
    for k in p:
        assert np.array_equal(p[k], q[k])
    assert M.flatten(p).size == 16 * 4 + 16 + 16 * 16 + 16 + 16 + 1
