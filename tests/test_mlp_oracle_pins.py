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


def test_splitmix64_matches_published_outputs():
    # the published first outputs of SplitMix64 seeded with 0
    from conftest import read_golden_lines

    exp = [int(x, 16) for x in read_golden_lines("splitmix64_seed0.txt")]
    assert [mlp.splitmix64(c) for c in range(len(exp))] == exp
    # a seeded stream continues the seed-0 stream: seed = k * gamma skips k outputs
    assert [mlp.splitmix64(c, seed=2 * 0x9E3779B97F4A7C15) for c in range(len(exp) - 2)] == exp[2:]


def test_sampled_pairs_are_distinct_and_cover_positions():
    k = 40
    pairs = [mlp.sampled_pair(7, t, k) for t in range(mlp.DENSITY_PAIRS)]
    assert all(0 <= a < b < k for a, b in pairs)
    # 256 draws over 40 positions: every position appears (a miss would point
    # at a biased mapping of the two halves of the output)
    assert {x for p in pairs for x in p} == set(range(k))
    # the mapping is uniform on ordered pairs: both orientations occur
    raw = [mlp.splitmix64(t, seed=mlp.splitmix64(7)) for t in range(mlp.DENSITY_PAIRS)]
    a = [(x & 0xFFFFFFFF) % k for x in raw]
    b = [(x >> 32) % (k - 1) for x in raw]
    assert any(bb >= aa for aa, bb in zip(a, b)) and any(bb < aa for aa, bb in zip(a, b))


def test_sampled_density_closed_forms_and_estimate():
    import oracle

    # K_30: P of the first root has 29 vertices (406 pairs > 256): every
    # sampled pair is adjacent, density exactly 1
    g = I.complete_graph(30)
    order, _ = oracle.sync_order(g)
    f = mlp.features(g, [int(order[0])], order)
    assert f[0, 3] == 1.0
    # star with 40 leaves: the centre's P (if it is a root with P) has no edges
    g = I.star_graph(40)
    order, _ = oracle.sync_order(g)
    f = mlp.features(g, list(range(g.n)), order)
    assert (f[:, 3] == 0).all()
    # Moon-Moser with 12 parts of 3: P of the first vertex is 33 vertices of
    # the other 11 parts, an exact density 1 - 11 * 3 / C(33, 2) = 0.9375; the
    # 256-pair estimate stays within 5 standard deviations of it
    g = I.moon_moser(12)
    order, _ = oracle.sync_order(g)
    v = int(order[0])
    f = mlp.features(g, [v], order)
    p = 1 - 11 * 3 / (33 * 32 / 2)
    sd = (p * (1 - p) / mlp.DENSITY_PAIRS) ** 0.5
    assert abs(f[0, 3] - p) <= 5 * sd
    assert f[0, 3] * mlp.DENSITY_PAIRS == round(f[0, 3] * mlp.DENSITY_PAIRS)  # a count of pairs


def _hand_theta():
    """A network whose hidden units are partly inactive on x = (1, 2, 0, 0):
    layer 1  z = (x0, -x0, x1 - 5, x1 + 0.5)            -> h = (1, 0, 0, 2.5)
    layer 2  z = (h0 + h1, h3 - 3, -h0 + h3)            -> h = (1, 0, 1.5)
    layer 3  z = (h0, h2 - h0, -h2)                     -> h = (1, 0.5, 0)
    output   y = 2 h0 + 4 h1 + 8 h2 + 0.25              =  4.25
    (every other weight and bias zero; mean 0, std 1)."""
    th = np.zeros(mlp.N_PARAMS)
    th[mlp.oStd:] = 1.0
    W1 = th[mlp.oW1:mlp.ob1].reshape(64, 4)
    b1 = th[mlp.ob1:mlp.oW2]
    W1[0, 0], W1[1, 0], W1[2, 1], W1[3, 1] = 1.0, -1.0, 1.0, 1.0
    b1[2], b1[3] = -5.0, 0.5
    W2 = th[mlp.oW2:mlp.ob2].reshape(64, 64)
    b2 = th[mlp.ob2:mlp.oW3]
    W2[0, 0], W2[0, 1] = 1.0, 1.0
    W2[1, 3], b2[1] = 1.0, -3.0
    W2[2, 0], W2[2, 3] = -1.0, 1.0
    W3 = th[mlp.oW3:mlp.ob3].reshape(64, 64)
    W3[0, 0] = 1.0
    W3[1, 2], W3[1, 0] = 1.0, -1.0
    W3[2, 2] = -1.0
    th[mlp.oW4:mlp.oW4 + 3] = [2.0, 4.0, 8.0]
    th[mlp.ob4] = 0.25
    return th


def test_forward_with_inactive_units_hand_computed():
    """Forward pass through units that ReLU switches off: the value worked out
    by hand in _hand_theta.  With ReLU replaced by the identity the same
    network gives z1 = (1,-1,-3,2.5), z2 = (0,-0.5,1.5), z3 = (0,1.5,-1.5) and
    y = -5.75, so the pin tells the two apart."""
    th = _hand_theta()
    y, c = mlp.forward(th, np.array([[1.0, 2.0, 0.0, 0.0]]))
    assert y[0] == 4.25
    assert list(c["h1"][0, :4]) == [1.0, 0.0, 0.0, 2.5]
    assert list(c["h2"][0, :3]) == [1.0, 0.0, 1.5]
    assert list(c["h3"][0, :3]) == [1.0, 0.5, 0.0]


def test_backward_through_inactive_units_hand_computed():
    """Loss (y - 0)^2 on the single sample above: dL/dy = 2 * 4.25 = 8.5.
    * dL/dW4 = 8.5 * h3 = (8.5, 4.25, 0);
    * units switched off pass no gradient: dL/db1[1] = dL/db1[2] = 0 and
      dL/db3[2] = 0;
    * dy/dh1[0]: through h2[0] (weight 1) into h3[0] (1, output 2) and h3[1]
      (-1, output 4) gives 2 - 4 = -2; through h2[2] (weight -1) into h3[1]
      (1, output 4) gives -4 (h3[2] is off); total -6, so dL/dW1[0,0] =
      8.5 * -6 * x0 = -51 and dL/db1[0] = -51;
    * dy/dh1[3]: through h2[1] (off) nothing; through h2[2] (weight 1) 4, so
      dL/dW1[3,1] = 8.5 * 4 * x1 = 68."""
    th = _hand_theta()
    loss, g = mlp.loss_grad(th, np.array([[1.0, 2.0, 0.0, 0.0]]), np.array([0.0]))
    assert loss == 4.25 ** 2
    assert list(g[mlp.oW4:mlp.oW4 + 3]) == [8.5, 4.25, 0.0]
    assert g[mlp.ob4] == 8.5
    gb1 = g[mlp.ob1:mlp.oW2]
    gW1 = g[mlp.oW1:mlp.ob1].reshape(64, 4)
    assert gb1[1] == 0.0 and gb1[2] == 0.0
    assert g[mlp.ob3 + 2] == 0.0
    assert gW1[0, 0] == -51.0 and gb1[0] == -51.0
    assert gW1[3, 1] == 68.0


def test_bf16_forward_exact_on_representable_network():
    """With BF16-exact weights and inputs and sums that FP32 holds exactly,
    the rounding-aware forward equals the plain forward and its radius is a
    few FP32 units."""
    th = _hand_theta()
    y, rad = mlp.forward_bf16(th, np.array([[1.0, 2.0, 0.0, 0.0]]))
    assert y[0] == 4.25
    assert rad[0] < 1e-4


def _fp32_bf16_forward(theta, X):
    """An independent FP32 evaluation (numpy float32 products and sums in
    BLAS order) with BF16 rounding at the same points."""
    p = mlp.unpack(theta)
    r = lambda a: mlp.bf16_round(a).astype(np.float32)  # noqa: E731
    X32 = np.asarray(X, dtype=np.float32)
    h = r((X32 - p["mean"].astype(np.float32)) / p["std"].astype(np.float32))
    for Wk, bk in (("W1", "b1"), ("W2", "b2"), ("W3", "b3")):
        z = h @ r(p[Wk]).T + r(p[bk])
        h = r(np.maximum(z, np.float32(0)))
    return (h @ r(p["W4"]) + np.float32(r(p["b4"]))).astype(np.float64)


@pytest.mark.parametrize("seed", range(3))
def test_bf16_forward_radius_covers_an_fp32_evaluation(seed):
    rng = np.random.default_rng(seed)
    th = _theta(seed, scale=0.4)
    th[mlp.oMean:mlp.oStd] = [2.0, 1.5, 5.0, 0.3]
    th[mlp.oStd:] = [1.0, 1.0, 2.0, 0.2]
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(4000, 4))
    y, rad = mlp.forward_bf16(th, X)
    y32 = _fp32_bf16_forward(th, X)
    assert (np.abs(y32 - y) <= rad).all()
    # the bound is informative: BF16 rounding makes it coarse only where an
    # activation sits on a rounding boundary
    scale = np.abs(y).max()
    assert np.median(rad) < 1e-3 * scale
    # and BF16 differs measurably from the FP64 network, which the radius
    # does not excuse
    y64, _ = mlp.forward(th, X)
    assert (np.abs(y64 - y) > rad).any()


@pytest.mark.parametrize("targets", ["random", "offset"])
def test_gradient_bound_covers_an_fp32_evaluation(targets):
    """loss_grad_bound: the FP32 gradient from an independent float32
    evaluation differs from the FP64 gradient by at most gamma(k) * A
    entry by entry (samples whose ReLU decisions rounding could flip are
    left out first).  The bound is a worst case: it takes every rounding
    error with the sign that adds up, through layers of mixed-sign weights, so
    it sits a few percent of an entry's magnitude above the FP64 value while
    actual FP32 errors are far smaller; it is used for its guarantee, next to
    a tighter aggregate check in the GPU test."""
    rng = np.random.default_rng(4)
    th = _theta(4, scale=0.3)
    X = rng.normal(size=(3000, 4)).astype(np.float32).astype(np.float64)
    if targets == "random":
        t = rng.normal(size=3000)
    else:
        t = mlp.forward(th, X)[0] - 1.0
    t = t.astype(np.float32).astype(np.float64)
    k = 1024
    _, _, margin = mlp.loss_grad_bound(th, X, t, k)
    keep = margin > 1.0
    X, t = X[keep], t[keep]
    A, A_loss, _ = mlp.loss_grad_bound(th, X, t, k)
    l64, g64 = mlp.loss_grad(th, X, t)
    # float32 evaluation of the same formulas
    p = {kk: v.astype(np.float32) if isinstance(v, np.ndarray) else np.float32(v)
         for kk, v in mlp.unpack(th).items()}
    X32, t32 = X.astype(np.float32), t.astype(np.float32)
    a0 = (X32 - p["mean"]) / p["std"]
    z1 = a0 @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0)
    z3 = h2 @ p["W3"].T + p["b3"]
    h3 = np.maximum(z3, 0)
    y = h3 @ p["W4"] + p["b4"]
    dy = np.float32(2) * (y - t32) / np.float32(len(t32))
    g = np.zeros(mlp.N_PARAMS, dtype=np.float32)
    g[mlp.oW4:mlp.ob4] = h3.T @ dy
    g[mlp.ob4] = dy.sum()
    d3 = np.outer(dy, p["W4"]) * (z3 > 0)
    g[mlp.oW3:mlp.ob3] = (d3.T @ h2).ravel()
    g[mlp.ob3:mlp.oW4] = d3.sum(0)
    d2 = (d3 @ p["W3"]) * (z2 > 0)
    g[mlp.oW2:mlp.ob2] = (d2.T @ h1).ravel()
    g[mlp.ob2:mlp.oW3] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (z1 > 0)
    g[mlp.oW1:mlp.ob1] = (d1.T @ a0).ravel()
    g[mlp.ob1:mlp.oW2] = d1.sum(0)
    bound = mlp.gamma(k) * A
    assert (np.abs(g.astype(np.float64) - g64) <= bound).all()
    # the bound is informative: a small fraction of each entry's magnitude
    nz = np.abs(g64) > 0
    assert np.median(bound[nz] / np.abs(g64[nz])) < 0.2
