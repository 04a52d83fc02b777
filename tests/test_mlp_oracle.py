"""Pins of the CPU oracle of the learned warm start (features, MLP forward,
backward, Adam, start vector) against facts independent of its code:
finite differences, closed forms and hand-computed positions."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo

SMALL = (6, 5, 4, 3, 2)


def test_bf16_rounding_known_values():
    x = np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-7, -2.0 - 2**-7 - 2**-9, 3.0e38, 0.0])
    got = mo.bf16_round(x)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to the even mantissa (1)
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == 1 + 2**-6 and got[3] == 1 + 2**-7
    assert got[4] == -(2.0 + 2**-6)   # ulp 2^-6 in [2, 4): above the half-way point
    assert np.isfinite(got[5]) and got[6] == 0.0


def _rand(seed, dims=SMALL, P=7):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.7, mo.param_count(dims))
    X = rng.normal(0, 1, (P, dims[0]))
    T = rng.normal(0, 1, (P, dims[-1]))
    return p, X, T


def _loss(p, X, T, dims):
    Y, _ = mo.forward(X, p, dims)
    return mo.mse(Y, T)[0]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_backward_matches_central_differences(seed):
    p, X, T = _rand(seed)
    Y, acts = mo.forward(X, p, SMALL)
    _, dY = mo.mse(Y, T)
    g = mo.backward(dY, acts, p, SMALL)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd[i] = (_loss(pp, X, T, SMALL) - _loss(pm, X, T, SMALL)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_forward_identity_network_is_relu():
    dims = (3, 3, 3, 3, 3)
    layers = [(np.eye(3), np.zeros(3)) for _ in range(4)]
    X = np.array([[1.0, -2.0, 0.5], [-1.0, 3.0, -0.25]])
    Y, acts = mo.forward(X, mo.pack(layers), dims)
    assert np.array_equal(Y, np.maximum(X, 0.0))
    assert len(acts) == 4 and np.array_equal(acts[0], X)


def test_bias_gradient_is_output_gradient_sum():
    p, X, T = _rand(5)
    Y, acts = mo.forward(X, p, SMALL)
    _, dY = mo.mse(Y, T)
    g = mo.unpack(mo.backward(dY, acts, p, SMALL), SMALL)
    assert np.allclose(g[-1][1], dY.sum(axis=0), rtol=0, atol=1e-15)
    assert np.allclose(g[-1][0], dY.T @ acts[-1], rtol=0, atol=1e-15)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p, g = rng.normal(size=10), rng.normal(size=10)
    z = np.zeros(10)
    p1, m1, v1 = mo.adam(p, g, z, z, 1, lr=0.01, eps=1e-8)
    # bias correction makes the first moments g and g^2 exactly (up to rounding)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_features_positions_masks_and_padding():
    batch, n = 2, 70          # two patches per system, the second one ragged
    arrs = [np.full((batch, n), 10.0 * (f + 1)) for f in range(7)]
    arrs[5] = np.arange(batch * n, dtype=float).reshape(batch, n)
    arrs[6] = np.zeros((batch, n))      # u_prev = 0: the residual feature is the rhs
    mean = np.array([1.0] * 7)
    scale = np.array([2.0] * 7)
    X = mo.features(*arrs, mean, scale)
    assert X.shape == (4, 448)
    # patch p = s * 2 + j; feature f at columns [64 f, 64 f + 64)
    assert X[3, 5 * 64 + 3] == (arrs[5][1, 64 + 3] - 1.0) / 2.0
    assert X[1, 5 * 64 + 6] == 0.0 and X[1, 5 * 64 + 5] == (arrs[5][0, 69] - 1.0) / 2.0
    assert X[0, 0] == (0.0 - 1.0) / 2.0 and X[0, 1] == -0.5 and X[0, 2] == (10.0 - 1) / 2
    assert X[0, 64] == -0.5 and X[0, 65] == (20.0 - 1) / 2                    # c_0
    assert X[1, 3 * 64 + 5] == -0.5 and X[1, 3 * 64 + 4] == (40.0 - 1) / 2   # a_{n-1}
    assert X[1, 4 * 64 + 4] == -0.5 and X[1, 4 * 64 + 3] == (50.0 - 1) / 2   # b_{n-2}


def test_residual_feature_of_exact_solution_is_zero():
    """Feature 5 is rhs - A u_prev: zero when u_prev solves the system, and
    the plain product otherwise (dense check)."""
    rng = np.random.default_rng(9)
    batch, n = 3, 130
    dg = [rng.normal(size=(batch, n)) for _ in range(5)]
    dg[2] += 6.0
    x = rng.normal(size=(batch, n))
    Ad = np.zeros((batch, n, n))
    for s in range(batch):
        for off, arr in zip((-2, -1, 0, 1, 2), dg):
            idx = np.arange(max(0, -off), min(n, n - off))
            Ad[s, idx, idx + off] = arr[s, idx]
    rhs = np.einsum("sij,sj->si", Ad, x)
    X = mo.features(*dg, rhs, x, np.zeros(7), np.ones(7))
    r = X[:, 5 * 64:6 * 64].reshape(batch, -1)[:, :n]
    assert np.abs(r).max() <= 1e-12 * np.abs(rhs).max()
    X2 = mo.features(*dg, rhs, np.zeros((batch, n)), np.zeros(7), np.ones(7))
    assert np.array_equal(X2[:, 5 * 64:6 * 64].reshape(batch, -1)[:, :n], rhs)


def test_apply_start_round_trip():
    rng = np.random.default_rng(4)
    batch, n = 3, 100
    x, up = rng.normal(size=(batch, n)), rng.normal(size=(batch, n))
    mu, sig = 0.25, 0.5
    Yp = np.zeros((batch * 2, 64))
    Yp.reshape(batch, 128)[:, :n] = (x - up - mu) / sig
    assert np.allclose(mo.apply_start(Yp, up, mu, sig), x, rtol=0, atol=1e-15)
