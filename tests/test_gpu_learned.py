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
        roots = np.arange(0, g.n, 3, dtype=np.int32)
        f = gpu_lib.root_features(dg, torch.from_numpy(roots).cuda()).cpu().numpy()
    # the later-neighbour sets P come from the oracle's own simulation of the
    # synchronous peel, not from the library's order
    order, _ = oracle.sync_order(g)
    exp = mlp.features(g, roots.tolist(), order)
    # FP32 log1p / division: a few units of FP32 rounding of values below 20
    assert np.allclose(f, exp, rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [1, 777, 9000])
def test_loss_grad_fp32_vs_fp64(gpu_lib, n):
    import torch

    rng = np.random.default_rng(n)
    th = _rand_model(n).astype(np.float64)
    # inputs and targets exactly representable in FP32, so both sides start
    # from the same numbers
    m_gen = 3 * n + 64  # about half the samples have a decision near zero
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(m_gen, 4))
    X = X.astype(np.float32).astype(np.float64)
    t = rng.normal(loc=3.0, size=m_gen).astype(np.float32).astype(np.float64)
    # Rounding bound: the FP32 kernels take at most K = 1024 roundings along
    # any chain of one gradient entry (forward: 4 + 2 x 64 per 64-input layer
    # and the output, about 400; backward through two 64-wide layers, about
    # 260; the weight-gradient sums over 64-sample tiles, 64 tiles per chunk
    # and the chunk partials, about 200), so |g - g_ref| <= gamma_K * A entry
    # by entry, A being the gradient with absolute values throughout.  The
    # bound needs equal ReLU decisions: samples with a pre-activation within
    # its rounding bound of zero are dropped first.
    K = 1024
    _, _, margin = mlp.loss_grad_bound(th, X, t, K)
    keep = np.flatnonzero(margin > 1.0)[:n]
    assert keep.size == n
    X, t = X[keep], t[keep]
    ref_loss, ref_g = mlp.loss_grad(th, X, t)
    A, A_loss, _ = mlp.loss_grad_bound(th, X, t, K)
    m = torch.from_numpy(th.astype(np.float32)).cuda()
    grad, loss = gpu_lib.model_loss_grad(m, torch.tensor(X, dtype=torch.float32).cuda(),
                                         torch.tensor(t, dtype=torch.float32).cuda())
    grad = grad.cpu().numpy().astype(np.float64)
    bound = mlp.gamma(K) * A
    bad = np.flatnonzero(np.abs(grad - ref_g) > bound)
    assert bad.size == 0, (bad[:5], grad[bad[:5]], ref_g[bad[:5]], bound[bad[:5]])
    assert abs(loss - ref_loss) <= mlp.gamma(K) * A_loss
    assert not grad[mlp.oMean:].any()
    # aggregate check, far tighter than the worst case: the rounding errors of
    # the entries do not all line up, so the error vector stays within 1e-4 of
    # the gradient's norm (observed ~1e-6)
    assert np.linalg.norm(grad - ref_g) <= 1e-4 * np.linalg.norm(ref_g)


def test_bf16_inference_within_rounding_bound(gpu_lib):
    import torch

    rng = np.random.default_rng(7)
    th = _rand_model(7)
    X = rng.normal(loc=[2.0, 1.5, 5.0, 0.3], scale=[1.0, 1.0, 2.0, 0.2], size=(5000, 4))
    X = X.astype(np.float32).astype(np.float64)
    # FP64 forward with the kernel's BF16 roundings (weights, biases, the
    # normalised input, every activation) and a radius covering any FP32
    # summation order; an activation whose interval reaches a BF16 rounding
    # boundary contributes one BF16 unit to the radius
    y_ref, rad = mlp.forward_bf16(th.astype(np.float64), X)
    y = gpu_lib.model_predict(torch.from_numpy(th).cuda(), torch.tensor(X, dtype=torch.float32).cuda())
    y = y.cpu().numpy().astype(np.float64)
    bad = np.flatnonzero(np.abs(y - y_ref) > rad)
    assert bad.size == 0, (bad[:5], y[bad[:5]], y_ref[bad[:5]], rad[bad[:5]])
    # the ranking the queue uses follows the FP64 network
    y64, _ = mlp.forward(th.astype(np.float64), X)
    assert np.corrcoef(y, y64)[0, 1] > 0.999


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
    # equal predictions: the target task is 1/workgroups of the total, so every
    # scored root (at least 16 later neighbours) becomes the same
    # ceil(workgroups / scored) groups (float rounding of the quotient may add
    # one when it is an integer) and every other root stays whole
    _, rank = oracle.sync_order(g)
    later = np.zeros(g.n, dtype=np.int64)
    for v in range(g.n):
        nb = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
        later[v] = int(np.count_nonzero(rank[nb] > rank[v]))
    scored = int(np.count_nonzero(later >= 16))
    n_roots = plain.stats["roots"]
    assert 0 < scored < plain.stats["workgroups"]
    extra = r.stats["roots"] - n_roots
    assert extra % scored == 0
    groups = -(-plain.stats["workgroups"] // scored)
    assert extra // scored + 1 in (min(groups, 64), min(groups + 1, 64))
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


def _list_schedule_makespan(cost, order, machines):
    """Greedy list scheduling: the roots in the given order, each to the
    machine that becomes free first (what a shared root counter does with
    equal workgroups and no donations); the largest finishing time."""
    import heapq

    free = [0.0] * machines
    for j in order:
        heapq.heapreplace(free, free[0] + float(cost[j]))
    return max(free)


def test_trained_model_gains_over_degeneracy_order(gpu_lib):
    """What the trained network gains over the method without it, measured on
    a held-out graph from the per-root tree-node counts of the plain run:
    recall of the heaviest 1% of roots among the first 1% of the queue, and
    the makespan of the queue under list scheduling, for degeneracy order
    (the plain queue), the out-degree heuristic and the model's order."""
    import torch
    from paper_2212_01473_amd import learned

    model = _trained_model(gpu_lib)
    g = I.rmat(15, 16, 0.57, 0.19, 0.19, 0.05, 97)
    n_nodes = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    cnt = torch.zeros_like(n_nodes)
    hsh = torch.zeros_like(n_nodes)
    with gpu_lib.load_graph(g) as dg:
        c = int(0.7 * dg.info().degeneracy)
        gpu_lib.enumerate_cliques(dg, max_root_core=c, root_stats=(cnt, hsh, n_nodes))
        core, _, order = dg.order_arrays()
        rank = np.empty(g.n, dtype=np.int64)
        rank[order] = np.arange(g.n)
        roots = order[(core[order] <= c)]
        src = np.repeat(np.arange(g.n), g.degrees())
        later = rank[g.col_idx.astype(np.int64)] > rank[src]
        outdeg = np.bincount(src[later], minlength=g.n)
        roots = roots[outdeg[roots] > 0]  # the queue: window roots with P non-empty, in degeneracy order
        feat = gpu_lib.root_features(dg, torch.from_numpy(roots.astype(np.int32)).cuda())
    pred = gpu_lib.model_predict(model, feat).cpu().numpy()
    cost = n_nodes.cpu().numpy()[roots].astype(np.float64)
    nr = len(roots)
    top = max(1, nr // 100)
    heavy = set(np.argsort(-cost, kind="stable")[:top].tolist())
    orders = {
        "degeneracy": np.arange(nr),
        "out_degree": np.argsort(-outdeg[roots], kind="stable"),
        "model": np.argsort(-pred, kind="stable"),
    }
    # the library's queue: roots with at least 16 later neighbours by the
    # model, then the others in degeneracy order
    scored = outdeg[roots] >= 16
    idx = np.arange(nr)
    orders["queue"] = np.concatenate([idx[scored][np.argsort(-pred[scored], kind="stable")], idx[~scored]])
    machines = 256
    lower = max(cost.sum() / machines, cost.max())
    recall = {k: len(heavy & set(o[:top].tolist())) / top for k, o in orders.items()}
    makespan = {k: _list_schedule_makespan(cost, o, machines) / lower for k, o in orders.items()}
    print(f"roots {nr}, top 1% = {top}: recall {recall}; makespan / lower bound {makespan}")
    assert recall["model"] > recall["degeneracy"]
    assert makespan["model"] < makespan["degeneracy"]
    assert makespan["queue"] < makespan["degeneracy"]
