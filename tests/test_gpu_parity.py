"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on the
same seeded inputs.  Count, histogram and hash must be bit-identical; the peel
arrays must equal the oracle's simulation of the synchronous peel."""
import ctypes as C
import itertools

import numpy as np
import pytest

import oracle
from paper_2212_01473_amd import inputs as I

pytestmark = pytest.mark.gpu

FULL = 0xFFFFFFFF


def _hist_dict(h):
    return {k: int(v) for k, v in enumerate(h) if v}


_ORACLE = {}


def oracle_result(g, c=FULL):
    key = (g.sha256(), c)
    if key not in _ORACLE:
        _ORACLE[key] = oracle.mce(g, max_root_core=c)
    return _ORACLE[key]


def check(mce, g, c=FULL, **kw):
    exp = oracle_result(g, c)
    with mce.load_graph(g) as dg:
        got = mce.enumerate_cliques(dg, max_root_core=c, timeout_ms=60000, **kw)
    assert got.count == exp.count, (g.name, kw)
    assert got.hash == exp.hash, (g.name, kw)
    assert _hist_dict(got.hist) == _hist_dict(exp.hist), (g.name, kw)
    return got, exp


# ---------------------------------------------------------------- small and closed forms

def test_fig1a(gpu_lib):
    got, _ = check(gpu_lib, I.fig1a_example())
    assert got.count == 2


@pytest.mark.parametrize("make", [
    lambda: I.complete_graph(1), lambda: I.complete_graph(2), lambda: I.complete_graph(7),
    lambda: I.complete_graph(64), lambda: I.complete_graph(65), lambda: I.complete_graph(130),
    lambda: I.empty_graph(1), lambda: I.empty_graph(33), lambda: I.moon_moser(4), lambda: I.moon_moser(8),
    lambda: I.cocktail_party(10), lambda: I.cycle_graph(3), lambda: I.cycle_graph(50), lambda: I.path_graph(40),
    lambda: I.star_graph(100), lambda: I.complete_multipartite([3, 5, 2, 7, 1]),
    lambda: I.disjoint_union([I.moon_moser(3), I.complete_graph(70), I.empty_graph(5), I.cycle_graph(9)]),
], ids=lambda f: "g")
def test_closed_forms(gpu_lib, make):
    check(gpu_lib, make())


def test_empty_vertex_set(gpu_lib):
    g = I.empty_graph(0)
    with gpu_lib.load_graph(g) as dg:
        r = gpu_lib.enumerate_cliques(dg)
    assert r.count == 0 and r.hash == 0


@pytest.mark.parametrize("seed", range(16))
def test_random_er(gpu_lib, seed):
    rng = np.random.default_rng(seed)
    if seed % 2:
        n = int(rng.integers(20, 70))
        p = float(rng.choice([0.3, 0.5, 0.7]))
    else:
        n = int(rng.integers(60, 2000))
        p = float(rng.choice([0.005, 0.02, 0.05, 0.1]))
    check(gpu_lib, I.erdos_renyi(n, p, 100 + seed))


def _dense(i):
    if i == 0:
        return I.complete_multipartite([2] * 8 + [1] * 114)   # 2^8 cliques of size 122
    if i == 1:
        return I.complete_multipartite([3] * 5 + [1] * 70)    # 3^5 cliques of size 75
    if i == 2:
        return I.chung_lu_planted(n=3000, wmax=30, n_cliques=12, cmin=70, cmax=100, pool=3000, seed=5)
    if i == 3:
        return I.complete_multipartite([2] * 6 + [1] * 250)   # 2^6 cliques of size 256
    return I.erdos_renyi(300, 0.5, 2100)


@pytest.mark.parametrize("i", range(5))
def test_dense_mid_mode(gpu_lib, i):
    """Universes above 64 vertices: bitmap rows of several words, re-indexing
    into the register form once P u X_P fits 64."""
    got, _ = check(gpu_lib, _dense(i))
    if i == 0:
        assert got.count == 256 and _hist_dict(got.hist) == {122: 256}


def test_er1000_workload(gpu_lib):
    got, exp = check(gpu_lib, I.workload("er1000"))
    assert exp.count == 8087


@pytest.mark.parametrize("scale", [10, 12, 13])
def test_rmat_full(gpu_lib, scale):
    check(gpu_lib, I.rmat(scale, 16, 0.57, 0.19, 0.19, 0.05, 50 + scale))


def test_rmat_windows(gpu_lib):
    g = I.rmat(14, 16, 0.57, 0.19, 0.19, 0.05, 2)
    core, _, _ = oracle.sync_peel(g)
    d = int(core.max())
    for c in (0, 1, 5, d // 3, d // 2):
        check(gpu_lib, g, c=c)


def test_chung_lu_planted_small(gpu_lib):
    g = I.chung_lu_planted(n=20000, wmax=200, n_cliques=60, cmin=20, cmax=60, pool=4000, seed=9)
    got, _ = check(gpu_lib, g)
    assert got.max_size >= 20


# ---------------------------------------------------------------- knobs never change results

@pytest.mark.parametrize("kw", [
    dict(worker_list=False),
    dict(donate_min_p=1),
    dict(donate_min_p=1, wg_per_cu=1),
    dict(bitmap_max_p=64),
    dict(bitmap_max_p=64, donate_min_p=2, wg_per_cu=2),
    dict(flags=0x40),  # reverse degeneracy order
    dict(donate_min_p=10, bitmap_max_p=256),  # the donation size of Section III-C
    dict(xrow_min_u=4096),  # no X rows: X_X as the partitioned index list with lookups
    dict(xrow_min_u=4096, donate_min_p=2, wg_per_cu=1),
    dict(xrow_ratio=1, bitmap_max_p=64),
])
def test_knobs_invariant(gpu_lib, kw):
    g = I.chung_lu_planted(n=8000, wmax=400, n_cliques=30, cmin=15, cmax=45, pool=300, seed=11)
    check(gpu_lib, g, **kw)
    check(gpu_lib, _dense(2), **kw)
    check(gpu_lib, _dense(4), **kw)


# ---------------------------------------------------------------- second-level subtrees (Algorithm 4)

@pytest.mark.parametrize("kw", [dict(), dict(worker_list=False), dict(donate_min_p=2, wg_per_cu=1),
                                dict(xrow_min_u=4096), dict(bitmap_max_p=64)])
def test_l2_roots_keep_results(gpu_lib, kw):
    graphs = [I.fig1a_example(), I.complete_graph(9), I.moon_moser(4), I.erdos_renyi(300, 0.08, 5), _dense(2),
              I.chung_lu_planted(n=8000, wmax=400, n_cliques=30, cmin=15, cmax=45, pool=300, seed=11)]
    for g in graphs:
        got, _ = check(gpu_lib, g, l2_roots=True, **kw)
    g = I.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, 3)
    for c in (8, 20, FULL):
        check(gpu_lib, g, c, l2_roots=True, **kw)


def test_l2_roots_reject_learned_order(gpu_lib):
    import torch

    from paper_2212_01473_amd import learned

    model = torch.from_numpy(learned.init_model(7)).cuda()
    with gpu_lib.load_graph(I.complete_graph(5)) as dg:
        with pytest.raises(gpu_lib.MCEError) as e:
            gpu_lib.enumerate_cliques(dg, l2_roots=True, model=model)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_ARG


def test_worker_list_donates(gpu_lib):
    # few workgroups, one heavy subtree: idle workgroups must receive branches
    got, _ = check(gpu_lib, _dense(4), donate_min_p=2, wg_per_cu=1)
    assert got.stats["donations"] > 0


@pytest.mark.parametrize("kw", [dict(), dict(xrow_min_u=4096)])
def test_fold_frames_carry_donations(gpu_lib, kw):
    # small universes: donated branches travel as register frames, which the
    # receiver runs without building bitmaps; without X rows only branches
    # with an empty X_X can fold
    g = I.chung_lu_planted(n=8000, wmax=400, n_cliques=30, cmin=15, cmax=45, pool=300, seed=11)
    got, _ = check(gpu_lib, g, donate_min_p=2, wg_per_cu=1, **kw)
    assert 0 < got.stats["fold_donations"] <= got.stats["donations"]


def test_custom_order(gpu_lib):
    import torch

    g = I.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, 8)
    perm = torch.tensor(np.random.default_rng(0).permutation(g.n).astype(np.int32), device="cuda")
    check(gpu_lib, g, root_order=perm)


def test_custom_order_rejects_non_permutations(gpu_lib):
    import torch

    g = I.rmat(10, 8, 0.57, 0.19, 0.19, 0.05, 8)
    bad_range = np.arange(g.n, dtype=np.int32)
    bad_range[5] = g.n
    dup = np.arange(g.n, dtype=np.int32)
    dup[7] = 3
    with gpu_lib.load_graph(g) as dg:
        for arr, msg in ((bad_range, "id >= n"), (dup, "not a permutation")):
            with pytest.raises(gpu_lib.MCEError) as e:
                gpu_lib.enumerate_cliques(dg, root_order=torch.from_numpy(arr).cuda())
            assert e.value.status == gpu_lib.MCE_ERR_INVALID_ARG and msg in str(e.value)
        # the handle still works after the rejected calls
        exp = oracle.mce(g)
        r = gpu_lib.enumerate_cliques(dg)
        assert (r.count, r.hash) == (exp.count, exp.hash)


def test_root_features_reject_bad_ids(gpu_lib):
    import torch

    g = I.rmat(10, 8, 0.57, 0.19, 0.19, 0.05, 8)
    with gpu_lib.load_graph(g) as dg:
        ids = torch.tensor([0, 1, g.n], dtype=torch.int32, device="cuda")
        with pytest.raises(gpu_lib.MCEError) as e:
            gpu_lib.root_features(dg, ids)
        assert e.value.status == gpu_lib.MCE_ERR_INVALID_ARG


# ---------------------------------------------------------------- peel arrays

@pytest.mark.parametrize("make", [lambda: I.workload("er1000"),
                                  lambda: I.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, 3),
                                  lambda: I.path_graph(300), lambda: I.fig1a_example()])
@pytest.mark.parametrize("peel_steps", [False, True], ids=["single_launch", "step_kernels"])
def test_peel_matches_sync_simulation(gpu_lib, make, peel_steps):
    g = make()
    core, rnd, nr = oracle.sync_peel(g)
    with gpu_lib.load_graph(g, peel_steps=peel_steps) as dg:
        gc, gr, order = dg.order_arrays()
        info = dg.info()
    # the single launch must be the one that ran (no silent fall back)
    assert info.peel_mode == (0 if g.n == 0 else 2 if peel_steps else 1)
    assert (gc == core).all()
    assert (gr == rnd).all()
    assert info.peel_rounds == nr
    assert info.degeneracy == int(core.max())
    exp_order = np.lexsort((np.arange(g.n), rnd))
    assert (order == exp_order).all()
    assert info.max_degree == int(g.degrees().max())


# ---------------------------------------------------------------- per-root statistics, stream

def test_root_stats_match_oracle_on_sampled_roots(gpu_lib):
    import torch

    g = I.rmat(13, 16, 0.57, 0.19, 0.19, 0.05, 21)
    cnt = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    hsh = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    nodes = torch.zeros(g.n, dtype=torch.int64, device="cuda")
    with gpu_lib.load_graph(g) as dg:
        r = gpu_lib.enumerate_cliques(dg, root_stats=(cnt, hsh, nodes))
    cnt = cnt.cpu().numpy().view(np.uint64)
    hsh = hsh.cpu().numpy().view(np.uint64)
    rng = np.random.default_rng(1)
    sample = rng.choice(g.n, size=200, replace=False)
    mask = np.zeros(g.n, dtype=np.uint8)
    mask[sample] = 1
    # a clique is reported by its earliest vertex, so attribute with the GPU's order
    sorder, _ = oracle.sync_order(g)
    exp = oracle.mce(g, root_mask=mask, order=sorder)
    iso = (g.degrees() == 0) & (mask == 1)
    assert int(cnt[sample].sum()) + int(iso.sum()) == exp.count
    h = (int(hsh[sample].sum(dtype=np.uint64)) + sum(oracle.clique_hash([v]) for v in np.flatnonzero(iso))) % 2**64
    assert h == exp.hash
    assert int(cnt.sum()) + int((g.degrees() == 0).sum()) == r.count


@pytest.mark.parametrize("case", ["er", "donated", "split"])
def test_stream_matches_oracle_cliques(gpu_lib, case):
    """The clique stream writes R from every executor: small universes, and
    (planted cliques of 70-100 vertices, forced donations, split roots) the mid,
    list and folded executors with R handed across donations and suspensions."""
    import torch

    kw = {}
    if case == "er":
        g = I.erdos_renyi(120, 0.3, 77)
    else:
        g = _dense(2)
        kw = dict(donate_min_p=2, wg_per_cu=1)
        if case == "split":
            from paper_2212_01473_amd import learned

            kw.update(model=torch.from_numpy(learned.init_model(3)).cuda(), split=True, split_top=64)
    exp = oracle.mce(g, collect=True)
    verts = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    offs = torch.zeros(1 << 14, dtype=torch.int64, device="cuda")
    with gpu_lib.load_graph(g) as dg:
        r = gpu_lib.enumerate_cliques(dg, stream_buffers=(verts, offs), **kw)
    assert r.status == 0
    if case == "donated":
        assert r.stats["donations"] > 0
    v = verts.cpu().numpy().view(np.uint32)
    o = offs.cpu().numpy().view(np.uint64)[: r.stream_cliques]
    got = sorted(tuple(sorted(int(x) for x in v[int(e >> 16): int(e >> 16) + int(e & 0xFFFF)])) for e in o)
    assert got == sorted(exp.cliques)


def test_stream_truncation_keeps_totals(gpu_lib):
    import torch

    g = I.erdos_renyi(120, 0.3, 78)
    exp = oracle.mce(g)
    verts = torch.zeros(50, dtype=torch.int32, device="cuda")
    offs = torch.zeros(10, dtype=torch.int64, device="cuda")
    with gpu_lib.load_graph(g) as dg:
        r = gpu_lib.enumerate_cliques(dg, stream_buffers=(verts, offs))
    assert r.status == gpu_lib.MCE_WARN_STREAM_TRUNCATED
    assert r.count == exp.count and r.hash == exp.hash


# ---------------------------------------------------------------- errors

def _bad_graphs():
    ok = I.cycle_graph(5)
    rp, ci = ok.row_ptr.astype(np.uint32), ok.col_idx.astype(np.uint32)
    asym = ci.copy(); asym[0] = 2           # row 0: {2, 4}, but row 2 lacks 0
    unsorted = ci.copy(); unsorted[[0, 1]] = unsorted[[1, 0]]
    selfloop = ci.copy(); selfloop[0] = 0
    oob = ci.copy(); oob[0] = 99
    dup = ci.copy(); dup[1] = dup[0]
    badrp = rp.copy(); badrp[2] = badrp[3] + 1
    # path 0-1-2 plus the arc 2 -> 0 alone: every arc v -> u with v < u has its
    # reverse, only a v > u arc lacks one (found by the arc counts)
    down_rp = np.array([0, 1, 3, 5], dtype=np.uint32)
    down_ci = np.array([1, 0, 2, 0, 1], dtype=np.uint32)
    # arcs 0-1 both ways, 2 -> 3 and 3 -> 1 without reverses: as many arcs go up
    # as down, but the two sets of pairs differ (found by the up-arc lookups)
    swap_rp = np.array([0, 1, 2, 3, 4], dtype=np.uint32)
    swap_ci = np.array([1, 0, 3, 1], dtype=np.uint32)
    return [(rp, asym), (rp, unsorted), (rp, selfloop), (rp, oob), (rp, dup), (badrp, ci), (down_rp, down_ci),
            (swap_rp, swap_ci)]


@pytest.mark.parametrize("i", range(8))
def test_invalid_graphs_rejected(gpu_lib, i):
    rp, ci = _bad_graphs()[i]
    with pytest.raises(gpu_lib.MCEError) as e:
        gpu_lib.load_csr(rp, ci)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_GRAPH
    assert "row" in str(e.value)


def _first_arc_without_reverse(rp, ci):
    """(row, position) of the first arc, in row-major order, whose reverse is
    missing; written with plain Python sets."""
    n = len(rp) - 1
    rows = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
    for v in range(n):
        for pos, u in enumerate(ci[rp[v]:rp[v + 1]].tolist()):
            if v not in rows[u]:
                return v, pos
    return None


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_asymmetric_with_equal_arc_counts_is_named(gpu_lib, seed):
    """One arc v -> u with u < v is removed and another arc b -> a with a < b is
    added: the numbers of arcs going up (to a larger id) and down stay equal,
    so only exact reverse lookups can reject the graph.  The message names the
    first offending arc in row-major order."""
    g = I.erdos_renyi(300, 0.05, 10 + seed)
    rng = np.random.default_rng(seed)
    rows = [list(g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    downs = [(v, u) for v in range(g.n) for u in rows[v] if u < v]
    v, u = downs[rng.integers(len(downs))]
    rows[v].remove(u)
    while True:
        a, b = sorted(int(x) for x in rng.choice(g.n, 2, replace=False))
        if a not in rows[b]:
            break
    rows[b] = sorted(rows[b] + [a])
    rp = np.zeros(g.n + 1, dtype=np.uint32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    ci = np.array([x for r in rows for x in r], dtype=np.uint32)
    up = sum(1 for x in range(g.n) for y in rows[x] if y > x)
    assert 2 * up == len(ci)  # as many arcs go up as down
    row, pos = _first_arc_without_reverse(rp, ci)
    with pytest.raises(gpu_lib.MCEError) as e:
        gpu_lib.load_csr(rp, ci)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_GRAPH
    assert f"asymmetric (missing reverse arc) at row {row} position {pos}" in str(e.value)


def test_hist_too_small(gpu_lib):
    g = I.complete_graph(9)
    with gpu_lib.load_graph(g) as dg:
        with pytest.raises(gpu_lib.MCEError) as e:
            gpu_lib.enumerate_cliques(dg, hist_len=5)
    assert e.value.status == gpu_lib.MCE_ERR_BUFFER_TOO_SMALL


def test_device_pointer_load(gpu_lib):
    import torch

    g = I.erdos_renyi(500, 0.05, 4)
    rp = torch.tensor(g.row_ptr.astype(np.int64), dtype=torch.int32, device="cuda")
    ci = torch.tensor(g.col_idx.astype(np.int64), dtype=torch.int32, device="cuda")
    exp = oracle.mce(g)
    with gpu_lib.load_csr(rp, ci) as dg:
        r = gpu_lib.enumerate_cliques(dg)
    assert (r.count, r.hash) == (exp.count, exp.hash)


def test_timeout_is_reported(gpu_lib):
    # a bounded watchdog set far below the run time: every wavefront must exit
    g = _dense(4)
    with gpu_lib.load_graph(g) as dg:
        with pytest.raises(gpu_lib.MCEError) as e:
            gpu_lib.enumerate_cliques(dg, timeout_ms=1)
        assert e.value.status == gpu_lib.MCE_ERR_TIMEOUT
        # the handle stays usable
        r = gpu_lib.enumerate_cliques(dg)
    exp = oracle_result(g)
    assert (r.count, r.hash) == (exp.count, exp.hash)


def test_batch_api(gpu_lib):
    graphs = [I.erdos_renyi(50 + 30 * i, 0.1 + 0.05 * i, i) for i in range(6)]
    with gpu_lib.load_batch(graphs) as dg:
        res = gpu_lib.enumerate_batch(dg)
        whole = dg.info(gpu_lib.GRAPH_WHOLE)
        members = [dg.info(i) for i in range(len(graphs))]
    # the whole-handle info describes the union
    assert whole.n_graphs == len(graphs) and whole.n == sum(g.n for g in graphs)
    assert whole.nnz == sum(len(g.col_idx) for g in graphs)
    assert whole.degeneracy == max(m.degeneracy for m in members)
    assert whole.max_degree == max(m.max_degree for m in members)
    exps = [oracle.mce(g) for g in graphs]
    for g, r, exp in zip(graphs, res, exps):
        assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist))
    # the result sequence: length, slices, negative indices and the array views agree
    assert len(res) == len(graphs)
    assert [r.count for r in res[1:4]] == [e.count for e in exps[1:4]]
    assert res[-1].hash == exps[-1].hash
    assert res.counts.tolist() == [e.count for e in exps]
    assert res.hashes.tolist() == [e.hash for e in exps]


def test_batch_with_a_large_member_peels_as_one_union(gpu_lib):
    # a member above the per-member peel's 8,192 vertices: the union peels as one
    # graph, with the same per-graph results
    graphs = [I.erdos_renyi(9000, 0.001, 3), I.complete_graph(12), I.erdos_renyi(200, 0.1, 4)]
    with gpu_lib.load_batch(graphs) as dg:
        res = gpu_lib.enumerate_batch(dg)
        assert dg.info().peel_mode in (1, 2)
        core, _, _ = dg.order_arrays(2)
    for g, r in zip(graphs, res):
        exp = oracle.mce(g)
        assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist))
    c2, _, _ = oracle.sync_peel(graphs[2])
    assert (core == c2).all()


def test_batch_union_matches_per_graph_oracle(gpu_lib):
    graphs = I.batch_graphs(count=48, seed=104, nmin=30, nmax=400)
    graphs.append(I.empty_graph(7))
    graphs.append(I.complete_graph(70))
    with gpu_lib.load_batch(graphs) as dg:
        res = gpu_lib.enumerate_batch(dg)
        info = [dg.info(i) for i in range(len(graphs))]
        core, rnd, order = dg.order_arrays(3)
        assert dg.info().peel_mode == 3
    for i, (g, r) in enumerate(zip(graphs, res)):
        exp = oracle_result(g)
        assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist)), i
        assert info[i].n == g.n and info[i].degeneracy == exp.degeneracy
    # every member peels on its own: its core numbers, rounds and order are those
    # of the oracle's simulation of its own synchronous peel
    c3, r3, _ = oracle.sync_peel(graphs[3])
    o3, _ = oracle.sync_order(graphs[3])
    assert (core == c3).all() and (rnd == r3).all()
    assert order.tolist() == o3.tolist()


def test_no_x_rows_variant(gpu_lib):
    # X rows disabled: every X_X test goes to the original graph
    check(gpu_lib, I.rmat(12, 16, 0.57, 0.19, 0.19, 0.05, 62), xrow_budget_words=1)
    check(gpu_lib, _dense(2), xrow_budget_words=1)


def _device_batch(graphs):
    import torch

    rp, ci, row_off, col_off = I.concat_batch(graphs)
    drp = torch.from_numpy(rp.astype(np.int64)).to(torch.int32).cuda()
    dci = torch.from_numpy((ci if ci.size else np.zeros(1, np.uint32)).astype(np.int64)).to(torch.int32).cuda()
    return drp, dci, row_off, col_off


def test_batch_device_pointers_match_host_load(gpu_lib):
    graphs = I.batch_graphs(count=40, seed=105, nmin=20, nmax=300)
    graphs.insert(5, I.empty_graph(3))
    drp, dci, row_off, col_off = _device_batch(graphs)
    with gpu_lib.load_batch_device(drp, dci, row_off, col_off) as dg:
        res = gpu_lib.enumerate_batch(dg)
    for i, (g, r) in enumerate(zip(graphs, res)):
        exp = oracle_result(g)
        assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist)), i


def test_batch_device_pointers_reject_bad_row_ptr(gpu_lib):
    graphs = [I.erdos_renyi(40, 0.2, s) for s in range(4)]
    drp, dci, row_off, col_off = _device_batch(graphs)
    # graph 2's last row pointer no longer equals its nnz
    drp[int(row_off[3]) - 1] -= 1
    with pytest.raises(gpu_lib.MCEError) as e:
        gpu_lib.load_batch_device(drp, dci, row_off, col_off)
    assert e.value.status == gpu_lib.MCE_ERR_INVALID_GRAPH and "graph 2" in str(e.value)


def test_autotune_keeps_results(gpu_lib):
    g = I.chung_lu_planted(n=6000, wmax=300, n_cliques=25, cmin=15, cmax=40, pool=300, seed=21)
    exp = oracle.mce(g)
    with gpu_lib.load_graph(g) as dg:
        opts, rep = gpu_lib.autotune(dg)
        assert rep["trials"] >= 1 + 3 + 2 + 2 + 1 + 2 and 0 < rep["best_ms"] <= rep["base_ms"]
        r = gpu_lib.enumerate_cliques(dg, options=opts)
    assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist))


def test_autotune_on_batch(gpu_lib):
    graphs = I.batch_graphs(count=24, seed=106, nmin=30, nmax=300)
    with gpu_lib.load_batch(graphs) as dg:
        opts, rep = gpu_lib.autotune(dg)
        res = gpu_lib.enumerate_batch(dg, options=opts)
    assert rep["best_ms"] <= rep["base_ms"]
    for i, (g, r) in enumerate(zip(graphs, res)):
        exp = oracle_result(g)
        assert (r.count, r.hash) == (exp.count, exp.hash), i


def test_batch_with_empty_and_vertexless_graphs(gpu_lib):
    """Members with no vertices or no edges sit between ordinary graphs; each
    member's results stay its own (host and device loaders)."""
    graphs = [I.empty_graph(0), I.complete_graph(5), I.empty_graph(4), I.empty_graph(0),
              I.erdos_renyi(60, 0.2, 9), I.empty_graph(0)]
    drp, dci, row_off, col_off = _device_batch(graphs)
    for load in (lambda: gpu_lib.load_batch(graphs), lambda: gpu_lib.load_batch_device(drp, dci, row_off, col_off)):
        with load() as dg:
            res = gpu_lib.enumerate_batch(dg)
            assert [dg.info(i).n for i in range(len(graphs))] == [g.n for g in graphs]
        for i, (g, r) in enumerate(zip(graphs, res)):
            exp = oracle_result(g)
            assert (r.count, r.hash, _hist_dict(r.hist)) == (exp.count, exp.hash, _hist_dict(exp.hist)), i
