"""Pins of the FP64 cost-model reference: finite differences for the
backward pass, a special case that reduces the network to a linear model
solved by least squares, the first Adam step, and feature definitions on
graphs with known structure."""
import numpy as np
import pytest

from oracle import mlp
from paper_2212_01473_amd import inputs as I


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-scale, scale, mlp.N_PARAMS)
    th[mlp.oMean:mlp.oStd] = 0.0
    th[mlp.oStd:] = 1.0
    return th


@pytest.mark.parametrize("seed", range(3))
def test_gradient_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    th = _theta(seed)
    X = rng.normal(size=(40, 4))
    t = rng.normal(size=40)
    _, g = mlp.loss_grad(th, X, t)
    idx = rng.choice(mlp.N_TRAINABLE, 60, replace=False)
    idx = np.concatenate([idx, [mlp.ob4, mlp.oW1, mlp.ob1, mlp.oW4]])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(th)
        e[i] = h
        fd = (mlp.loss(th + e, X, t) - mlp.loss(th - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i
    assert not g[mlp.oMean:].any()


def test_linear_special_case_reduces_to_least_squares():
    """With non-negative inputs and non-negative identity-like weights every ReLU
    is active, so y = c . x + d; the MSE gradient w.r.t. (c, d) of a linear
    model is the normal-equation residual, checked through numpy lstsq."""
    rng = np.random.default_rng(5)
    X = rng.uniform(0.5, 2.0, size=(30, 4))
    th = np.zeros(mlp.N_PARAMS)
    th[mlp.oStd:] = 1.0
    W1 = th[mlp.oW1:mlp.ob1].reshape(64, 4)
    W1[:4, :] = np.eye(4)
    W2 = th[mlp.oW2:mlp.ob2].reshape(64, 64)
    W3 = th[mlp.oW3:mlp.ob3].reshape(64, 64)
    W2[:4, :4] = np.eye(4)
    W3[:4, :4] = np.eye(4)
    c = np.array([0.5, -0.25, 1.0, 2.0])
    th[mlp.oW4:mlp.oW4 + 4] = c
    th[mlp.ob4] = 0.3
    y, _ = mlp.forward(th, X)
    assert np.allclose(y, X @ c + 0.3)
    # the least-squares optimum has zero gradient w.r.t. the last layer
    t = rng.normal(size=30)
    A = np.hstack([X, np.ones((30, 1))])
    sol, *_ = np.linalg.lstsq(A, t, rcond=None)
    th2 = th.copy()
    th2[mlp.oW4:mlp.oW4 + 4] = sol[:4]
    th2[mlp.ob4] = sol[4]
    _, g = mlp.loss_grad(th2, X, t)
    assert np.abs(g[mlp.oW4:mlp.oW4 + 4]).max() < 1e-10
    assert abs(g[mlp.ob4]) < 1e-10


def test_first_adam_step_moves_by_lr_times_sign():
    rng = np.random.default_rng(2)
    th = _theta(2)
    g = rng.normal(size=mlp.N_PARAMS)
    opt = mlp.Adam(lr=0.01, eps=1e-12)
    th2 = opt.step(th, g)
    d = th2[:mlp.N_TRAINABLE] - th[:mlp.N_TRAINABLE]
    assert np.allclose(d, -0.01 * np.sign(g[:mlp.N_TRAINABLE]), atol=1e-9)
    assert (th2[mlp.oMean:] == th[mlp.oMean:]).all()


def test_fit_norm_standardises():
    rng = np.random.default_rng(3)
    X = rng.normal(loc=[1, 2, 3, 4], scale=[1, 2, 3, 4], size=(500, 4))
    th = mlp.fit_norm(_theta(0), X)
    y, c = mlp.forward(th, X)
    assert np.allclose(c["a0"].mean(0), 0, atol=1e-12)
    assert np.allclose(c["a0"].std(0), 1, atol=1e-12)


def test_features_closed_forms():
    import oracle

    # complete graph K_n: the first root in any order has P = n-1 vertices, density 1
    g = I.complete_graph(9)
    order, _ = oracle.sync_order(g)
    f = mlp.features(g, [int(order[0])], order)
    assert np.isclose(f[0, 0], np.log1p(8)) and np.isclose(f[0, 1], np.log1p(8))
    assert np.isclose(f[0, 2], np.log1p(8 * 8)) and np.isclose(f[0, 3], 1.0)
    # star: the centre's later neighbours are pairwise non-adjacent
    g = I.star_graph(10)
    order, _ = oracle.sync_order(g)
    f = mlp.features(g, list(range(g.n)), order)
    assert (f[:, 3] == 0).all()
    # Moon-Moser: later neighbours of the first vertex form MM minus its part
    g = I.moon_moser(3)
    order, _ = oracle.sync_order(g)
    v = int(order[0])
    f = mlp.features(g, [v], order)
    # P = the 6 vertices of the other two parts: 3*3 edges among C(6,2) = 15 pairs
    assert np.isclose(f[0, 3], 9 / 15)
