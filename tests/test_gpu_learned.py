"""GPU checks of the learned root ordering: features and FP32 gradients against
the FP64 reference, BF16 inference within its rounding bound, GPU training
against the reference optimiser, and enumeration results unchanged by the
learned order and split."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2212_01473_amd import inputs as I

pytestmark = pytest.mark.gpu


def _hist_dict(h):
    return {k: int(v) for k, v in enumerate(h) if v}


def _rand_model(seed):
    from paper_2212_01473_amd import learned

    th = learned.init_model(seed)
    rng = np.random.default_rng(seed)
    th[mlp.ob1:mlp.oW2] = rng.uniform(0.0, 0.2, 64)  # keep some units active
    th[mlp.ob2:mlp.oW3] = rng.uniform(0.0, 0.2, 64)
    th[mlp.ob3:mlp.oW4] = rng.uniform(0.0, 0.2, 64)
    th[mlp.oMean:mlp.oStd] = [2.0, 1.5, 5.0, 0.3]
    th[mlp.oStd:] = [1.0, 1.0, 2.0, 0.2]
    return th


def test_features_match_reference(gpu_lib):
    import torch

    g = I.rmat(11, 16, 0.57, 0.19, 0.19, 0.05, 31)
    with gpu_lib.load_graph(g) as dg:
        _, _, order = dg.order_arrays()
        roots = np.arange(0, g.n, 3, dtype=np.int32)
        f = gpu_lib.root_features(dg, torch.from_numpy(roots).cuda()).cpu().numpy()
    exp = mlp.features(g, roots.tolist(), order)
    assert np.allclose(f, exp, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [1, 777, 9000])
def test_loss_grad_fp32_vs_fp64(gpu_lib, n):
    import torch

    rng = np.random.default_rng(n)
    th = _rand_model(n)
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(n, 4))
    t = rng.normal(loc=3.0, size=n)
    ref_loss, ref_g = mlp.loss_grad(th.astype(np.float64), X, t)
    m = torch.from_numpy(th).cuda()
    grad, loss = gpu_lib.model_loss_grad(m, torch.tensor(X, dtype=torch.float32).cuda(),
                                         torch.tensor(t, dtype=torch.float32).cuda())
    grad = grad.cpu().numpy().astype(np.float64)
    # FP32 sums of n terms: relative error of the gradient vector <= 1e-4
    assert np.linalg.norm(grad - ref_g) <= 1e-4 * np.linalg.norm(ref_g) + 1e-7
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss + 1e-7
    assert not grad[mlp.oMean:].any()


def test_bf16_inference_within_rounding_bound(gpu_lib):
    import torch

    rng = np.random.default_rng(7)
    th = _rand_model(7)
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(5000, 4))
    y_ref, _ = mlp.forward(th.astype(np.float64), X)
    y = gpu_lib.model_predict(torch.from_numpy(th).cuda(), torch.tensor(X, dtype=torch.float32).cuda())
    y = y.cpu().numpy()
    # bf16 keeps 8 significant bits (relative rounding <= 2^-9 per value); through
    # four layers of sums of 64 products the error stays below 3% of the scale
    scale = np.abs(y_ref).max() + 1.0
    assert np.abs(y - y_ref).max() <= 0.03 * scale
    assert np.corrcoef(y, y_ref)[0, 1] > 0.999


def test_gpu_training_follows_reference_adam(gpu_lib):
    import torch

    rng = np.random.default_rng(11)
    th0 = _rand_model(11)
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(3000, 4))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 2] + rng.normal(scale=0.05, size=3000)
    m = torch.from_numpy(th0.copy()).cuda()
    hist = gpu_lib.model_train(m, torch.tensor(X, dtype=torch.float32).cuda(),
                               torch.tensor(t, dtype=torch.float32).cuda(), epochs=30, lr=1e-3, fit_norm=False)
    th = th0.astype(np.float64)
    opt = mlp.Adam(lr=1e-3)
    ref = []
    for _ in range(30):
        l, g = mlp.loss_grad(th, X, t)
        ref.append(l)
        th = opt.step(th, g)
    assert np.allclose(hist, ref, rtol=2e-3)
    got = m.cpu().numpy().astype(np.float64)
    assert np.abs(got - th).max() < 5e-4
    assert hist[-1] < hist[0]


def _trained_model(gpu_lib, seed=0):
    import torch
    from paper_2212_01473_amd import learned

    g = I.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, 41)
    feat, label = learned.collect(g, 60)
    model, hist = learned.train(feat, label, epochs=200, seed=seed)
    assert hist[-1] < hist[0]
    return model


@pytest.mark.parametrize("split", [False, True])
def test_learned_order_keeps_results(gpu_lib, split):
    import torch

    model = _trained_model(gpu_lib)
    rand = torch.from_numpy(_rand_model(3)).cuda()
    for g, c in ((I.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, 17), 0xFFFFFFFF),
                 (I.rmat(14, 16, 0.57, 0.19, 0.19, 0.05, 2), 60),
                 (I.chung_lu_planted(n=8000, wmax=400, n_cliques=30, cmin=15, cmax=45, pool=300, seed=11),
                  0xFFFFFFFF)):
        exp = oracle.mce(g, max_root_core=c)
        with gpu_lib.load_graph(g) as dg:
            plain_roots = gpu_lib.enumerate_cliques(dg, max_root_core=c).stats["roots"]
            for m in (model, rand):
                r = gpu_lib.enumerate_cliques(dg, max_root_core=c, model=m, split=split, timeout_ms=60000)
                assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist))
                if split:
                    assert r.stats["tasks"] >= r.stats["roots"]
                    if m is model:
                        # the costliest roots by rank are split into 64 groups each
                        assert r.stats["roots"] >= plain_roots + 63
                else:
                    assert r.stats["roots"] == plain_roots


def test_split_every_root_keeps_results(gpu_lib):
    import torch

    rand = torch.from_numpy(_rand_model(5)).cuda()
    # zero output weights and a huge bias: every root is predicted equally costly
    rand[mlp.oW4:mlp.ob4] = 0.0
    rand[mlp.ob4] = 30.0
    g = I.chung_lu_planted(n=3000, wmax=30, n_cliques=12, cmin=70, cmax=100, pool=3000, seed=5)
    exp = oracle.mce(g)
    with gpu_lib.load_graph(g) as dg:
        plain = gpu_lib.enumerate_cliques(dg, timeout_ms=60000)
        r = gpu_lib.enumerate_cliques(dg, model=rand, split=True, timeout_ms=60000)
    assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist))
    # equal predictions: the target task is 1/(4 * workgroups) of the total, so
    # every root becomes the same ceil(4 * workgroups / roots) groups (float
    # rounding of the quotient may add one when it is an integer)
    n_roots = plain.stats["roots"]
    assert r.stats["roots"] % n_roots == 0
    groups = -(-4 * plain.stats["workgroups"] // n_roots)
    assert r.stats["roots"] // n_roots in (min(groups, 64), min(groups + 1, 64))
    assert r.stats["roots"] > n_roots


def test_trained_model_ranks_held_out_roots(gpu_lib):
    """The model trained on one graph orders the roots of another by cost:
    Spearman correlation between predicted and measured cost."""
    import torch
    from paper_2212_01473_amd import learned

    model = _trained_model(gpu_lib)
    g = I.rmat(14, 16, 0.57, 0.19, 0.19, 0.05, 99)
    feat, label = learned.collect(g, 80)
    pred = gpu_lib.model_predict(model, feat).cpu().numpy()
    lab = label.cpu().numpy()
    rp = np.argsort(np.argsort(pred))
    rl = np.argsort(np.argsort(lab))
    rho = np.corrcoef(rp, rl)[0, 1]
    assert rho > 0.6, rho
