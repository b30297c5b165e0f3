"""Seeded synthetic graph generators.

This module produces the inputs that both the HIP path and the CPU oracle
consume.  It holds none of the enumeration method's arithmetic: no ordering,
no core numbers, no cliques.  It only draws random edges and puts them in the
canonical form the library accepts (simple undirected graph, uint32 CSR,
symmetric, rows strictly increasing, no self-loops).

Generator recipes (one per workload):

* ``erdos_renyi(n, p, seed)``: i.i.d. Bernoulli(p) on every pair i<j.
* ``rmat(scale, edge_factor, a, b, c, d, seed)``: 2^scale * edge_factor
  samples; each of the ``scale`` bits of an edge picks one quadrant from one
  uniform draw (u<a -> (0,0), u<a+b -> (0,1), u<a+b+c -> (1,0), else (1,1)),
  most significant bit first.  No noise, no permutation.  Self-loops and
  duplicates dropped, symmetrised.
* ``chung_lu_planted(...)``: weights from a continuous power law by inverse
  CDF, the largest forced to the stated maximum; M = round(sum(w)/2) edges with
  both endpoints drawn in proportion to w; plus planted cliques whose members
  are drawn without replacement from the highest-weight vertices.
* ``batch_graphs(count, seed)``: per-graph child seeds from
  ``SeedSequence(seed).spawn(count)``; n log-uniform in [50, 5000]; even index
  Erdos-Renyi with average degree U[5, 40]; odd index planted partition with 8
  contiguous near-equal blocks, p_in = 0.3, p_out = 0.005.
* Closed-form families (complete, empty, Moon-Moser, complete multipartite,
  cocktail party, cycle, path, star) and the six-vertex example graph of the
  paper's background section (Fig. 1(a): maximal cliques ABCD and AEF).

All random numbers come from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import hashlib
import math
import os
from dataclasses import dataclass

import numpy as np


@dataclass
class CSRGraph:
    """Undirected simple graph in uint32 CSR form (both arc directions stored)."""

    n: int
    row_ptr: np.ndarray  # uint32[n+1] (uint64 when nnz >= 2^32)
    col_idx: np.ndarray  # uint32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.uint64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr).tobytes())
        h.update(np.ascontiguousarray(self.col_idx).tobytes())
        return h.hexdigest()

    def edges(self) -> np.ndarray:
        """Edge list (u < v), int64[m, 2]."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col_idx.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, np.random.SeedSequence):
        return np.random.Generator(np.random.PCG64(seed))
    return np.random.Generator(np.random.PCG64(int(seed)))


def from_edges(n: int, src, dst, name: str = "") -> CSRGraph:
    """Canonical CSR from an arbitrary arc list: drop self-loops, symmetrise,
    remove duplicates, sort every row."""
    src = np.asarray(src, dtype=np.int64).ravel()
    dst = np.asarray(dst, dtype=np.int64).ravel()
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("vertex id out of range")
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    del key
    a = np.concatenate([lo, hi])
    b = np.concatenate([hi, lo])
    del lo, hi
    order = np.lexsort((b, a))
    a = a[order]
    b = b[order]
    counts = np.bincount(a, minlength=n).astype(np.int64)
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rp[1:])
    rp_dtype = np.uint32 if rp[-1] < 2**32 else np.uint64
    return CSRGraph(n=n, row_ptr=rp.astype(rp_dtype), col_idx=b.astype(np.uint32), name=name)


def from_adjacency_lists(adj: dict | list, n: int | None = None, name: str = "") -> CSRGraph:
    if isinstance(adj, dict):
        n = n if n is not None else (max(adj) + 1 if adj else 0)
        items = adj.items()
    else:
        n = len(adj) if n is None else n
        items = enumerate(adj)
    src, dst = [], []
    for u, nbrs in items:
        for v in nbrs:
            src.append(u)
            dst.append(v)
    return from_edges(n, src, dst, name)


# ---------------------------------------------------------------- closed forms

def empty_graph(n: int) -> CSRGraph:
    return from_edges(n, [], [], f"empty{n}")


def complete_graph(n: int) -> CSRGraph:
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju, f"K{n}")


def complete_multipartite(sizes) -> CSRGraph:
    sizes = [int(s) for s in sizes]
    part = np.repeat(np.arange(len(sizes)), sizes)
    n = int(sum(sizes))
    iu, ju = np.triu_indices(n, 1)
    keep = part[iu] != part[ju]
    return from_edges(n, iu[keep], ju[keep], "K_" + "_".join(map(str, sizes)))


def moon_moser(k: int) -> CSRGraph:
    """Complete k-partite graph with parts {3i, 3i+1, 3i+2}."""
    g = complete_multipartite([3] * k)
    g.name = f"MM{k}"
    return g


def cocktail_party(k: int) -> CSRGraph:
    g = complete_multipartite([2] * k)
    g.name = f"CP{k}"
    return g


def cycle_graph(n: int) -> CSRGraph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, f"C{n}")


def path_graph(n: int) -> CSRGraph:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1, f"P{n}")


def star_graph(m: int) -> CSRGraph:
    return from_edges(m + 1, np.zeros(m, dtype=np.int64), np.arange(1, m + 1), f"S{m}")


def disjoint_union(graphs) -> CSRGraph:
    src, dst, off = [], [], 0
    for g in graphs:
        e = g.edges()
        src.append(e[:, 0] + off)
        dst.append(e[:, 1] + off)
        off += g.n
    if not src:
        return empty_graph(0)
    return from_edges(off, np.concatenate(src), np.concatenate(dst), "union")


def fig1a_example() -> CSRGraph:
    """Six-vertex example of the background section (Fig. 1(a)): A..F -> 0..5,
    maximal cliques ABCD and AEF, so A has degree 5.  The edge set is forced by
    those two facts: the six edges inside ABCD plus AE, AF and EF."""
    A, B, C, D, E, F = range(6)
    edges = [(A, B), (A, C), (A, D), (B, C), (B, D), (C, D), (A, E), (A, F), (E, F)]
    s, t = zip(*edges)
    return from_edges(6, s, t, "fig1a")


def random_graph_from_mask(n: int, mask: int) -> CSRGraph:
    """Graph on n vertices whose edge (i<j) is present iff bit k of ``mask`` is
    set, pairs enumerated in row-major order of the strict upper triangle."""
    iu, ju = np.triu_indices(n, 1)
    bits = np.array([(mask >> k) & 1 for k in range(iu.size)], dtype=bool)
    return from_edges(n, iu[bits], ju[bits], f"mask{n}_{mask}")


# ---------------------------------------------------------------- random families

def _bernoulli_positions(rng: np.random.Generator, count: int, p: float) -> np.ndarray:
    """Indices in [0, count) of successes of ``count`` i.i.d. Bernoulli(p)
    trials, drawn by geometric gaps (exact for any p)."""
    if count <= 0 or p <= 0.0:
        return np.zeros(0, dtype=np.int64)
    if p >= 1.0:
        return np.arange(count, dtype=np.int64)
    if p > 0.2:
        return np.flatnonzero(rng.random(count) < p).astype(np.int64)
    out = []
    pos = -1
    while True:
        need = int(max(64, (count - pos) * p * 1.1 + 6 * math.sqrt((count - pos) * p + 1)))
        gaps = rng.geometric(p, size=need).astype(np.int64)
        cs = pos + np.cumsum(gaps)
        inside = cs[cs < count]
        out.append(inside)
        if inside.size < cs.size:
            break
        pos = int(cs[-1])
    return np.concatenate(out)


def _triu_pair(n: int, k: np.ndarray):
    """Map row-major strict-upper-triangle index k to (i, j), i < j < n."""
    k = k.astype(np.int64)
    # row i starts at s(i) = i*n - i*(i+1)/2
    nf = float(n)
    i = np.floor(((2 * nf - 1) - np.sqrt((2 * nf - 1) ** 2 - 8.0 * k)) / 2).astype(np.int64)
    i = np.clip(i, 0, max(n - 2, 0))
    start = i * n - i * (i + 1) // 2
    # fix rounding
    over = k < start
    while over.any():
        i[over] -= 1
        start = i * n - i * (i + 1) // 2
        over = k < start
    nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
    under = k >= nxt
    while under.any():
        i[under] += 1
        nxt = (i + 1) * n - (i + 1) * (i + 2) // 2
        under = k >= nxt
    start = i * n - i * (i + 1) // 2
    j = k - start + i + 1
    return i, j


def erdos_renyi(n: int, p: float, seed) -> CSRGraph:
    """G(n, p): every pair i<j (row-major order) present with probability p."""
    rng = _rng(seed)
    npairs = n * (n - 1) // 2
    if npairs <= 4_000_000:
        hit = np.flatnonzero(rng.random(npairs) < p)
    else:
        hit = _bernoulli_positions(rng, npairs, p)
    i, j = _triu_pair(n, hit)
    return from_edges(n, i, j, f"er{n}_{p}")


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, d: float, seed,
         chunk: int = 1 << 24, workers: int = 8) -> CSRGraph:
    """R-MAT: n = 2^scale vertices, edge_factor * n samples; per sample and bit
    (most significant first) one uniform u picks the quadrant (u < a: (0,0),
    < a+b: (0,1), < a+b+c: (1,0), else (1,1)).  Self-loops and duplicates are
    dropped and the graph is symmetrised.

    The samples are drawn in chunks of `chunk`, each chunk bit by bit from one
    PCG64 stream; chunks run in threads, each starting from the stream advanced
    to its first draw, and the arcs are deduplicated in row-range buckets, so
    the graph does not depend on `workers`."""
    n = 1 << scale
    m = n * edge_factor
    thr = np.array([a, a + b, a + b + c])
    nb = max(1, int(workers))
    rows_per = (n + nb - 1) // nb
    bounds = np.array([min(n, (i + 1) * rows_per) * n for i in range(nb - 1)], dtype=np.int64)

    def sample(start):
        k = min(chunk, m - start)
        rng = _rng(seed)
        rng.bit_generator.advance(start * scale)  # one 64-bit draw per uniform
        s = np.zeros(k, dtype=np.int64)
        t = np.zeros(k, dtype=np.int64)
        for bit in range(scale - 1, -1, -1):
            q = np.searchsorted(thr, rng.random(k), side="right")  # quadrant 0..3
            s |= (q >> 1) << bit
            t |= (q & 1) << bit
        keep = s != t
        s, t = s[keep], t[keep]
        arcs = np.unique(np.concatenate([s * n + t, t * n + s]))  # row * n + col, both directions
        return np.split(arcs, np.searchsorted(arcs, bounds))

    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(nb) as ex:
        parts = list(ex.map(sample, range(0, m, chunk)))
        merged = list(ex.map(lambda i: np.unique(np.concatenate([p[i] for p in parts])), range(nb)))
    del parts
    arcs = np.concatenate(merged)
    del merged
    row = arcs // n
    col = (arcs - row * n).astype(np.uint32)
    del arcs
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(row, minlength=n), out=rp[1:])
    rp_dtype = np.uint32 if rp[-1] < 2**32 else np.uint64
    return CSRGraph(n=n, row_ptr=rp.astype(rp_dtype), col_idx=col, name=f"rmat{scale}_ef{edge_factor}")


def chung_lu_planted(n: int = 1_000_000, exponent: float = 2.1, wmin: float = 2.0,
                     wmax: float = 5000.0, n_cliques: int = 2000, cmin: int = 20,
                     cmax: int = 60, pool: int = 20000, seed=3) -> CSRGraph:
    rng = _rng(seed)
    e = 1.0 - exponent
    lo, hi = wmin ** e, wmax ** e
    u = rng.random(n)
    w = (lo - u * (lo - hi)) ** (1.0 / e)
    w[int(np.argmax(w))] = wmax
    M = int(round(w.sum() / 2.0))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    src = np.searchsorted(cdf, rng.random(M), side="right")
    dst = np.searchsorted(cdf, rng.random(M), side="right")
    src = np.minimum(src, n - 1)
    dst = np.minimum(dst, n - 1)
    top = np.argsort(-w, kind="stable")[:pool]
    ps, pd = [src.astype(np.int64)], [dst.astype(np.int64)]
    for _ in range(n_cliques):
        size = int(rng.integers(cmin, cmax + 1))
        members = rng.choice(top, size=size, replace=False).astype(np.int64)
        iu, ju = np.triu_indices(size, 1)
        ps.append(members[iu])
        pd.append(members[ju])
    return from_edges(n, np.concatenate(ps), np.concatenate(pd), f"chunglu{n}")


def planted_partition(n: int, blocks: int, p_in: float, p_out: float, seed) -> CSRGraph:
    rng = _rng(seed)
    bounds = [(n * i) // blocks for i in range(blocks + 1)]
    srcs, dsts = [], []
    for bi in range(blocks):
        a0, a1 = bounds[bi], bounds[bi + 1]
        na = a1 - a0
        # inside block bi: pairs of the strict upper triangle
        hit = _bernoulli_positions(rng, na * (na - 1) // 2, p_in)
        i, j = _triu_pair(na, hit) if hit.size else (hit, hit)
        srcs.append(i + a0)
        dsts.append(j + a0)
        for bj in range(bi + 1, blocks):
            b0, b1 = bounds[bj], bounds[bj + 1]
            nb = b1 - b0
            hit = _bernoulli_positions(rng, na * nb, p_out)
            srcs.append(hit // nb + a0)
            dsts.append(hit % nb + b0)
    return from_edges(n, np.concatenate(srcs), np.concatenate(dsts), f"pp{n}")


def batch_graph_spec(index: int, child: np.random.SeedSequence, nmin: int = 50, nmax: int = 5000):
    rng = _rng(child)
    n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
    if index % 2 == 0:
        k = float(rng.uniform(5.0, 40.0))
        p = min(1.0, k / max(n - 1, 1))
        return ("er", n, p, rng)
    return ("pp", n, None, rng)


def batch_graphs(count: int = 4096, seed: int = 4, nmin: int = 50, nmax: int = 5000):
    """The batched workload: ``count`` independent graphs of uneven sizes."""
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for idx, ch in enumerate(children):
        kind, n, p, rng = batch_graph_spec(idx, ch, nmin, nmax)
        sub = np.random.SeedSequence(int(rng.integers(0, 2**63 - 1)))
        if kind == "er":
            g = erdos_renyi(n, p, sub)
        else:
            g = planted_partition(n, 8, 0.3, 0.005, sub)
        g.name = f"batch{seed}_{idx}_{kind}{n}"
        out.append(g)
    return out


def concat_batch(graphs):
    """Concatenate CSRs for the batch loader: per-graph row_ptr arrays (each
    starting at 0) laid end to end, plus uint64 offsets into both arrays."""
    row_off = np.zeros(len(graphs) + 1, dtype=np.uint64)
    col_off = np.zeros(len(graphs) + 1, dtype=np.uint64)
    for i, g in enumerate(graphs):
        row_off[i + 1] = row_off[i] + np.uint64(g.n + 1)
        col_off[i + 1] = col_off[i] + np.uint64(g.nnz)
    rp = np.concatenate([g.row_ptr.astype(np.uint32) for g in graphs]) if graphs else np.zeros(0, np.uint32)
    ci = np.concatenate([g.col_idx for g in graphs]) if graphs else np.zeros(0, np.uint32)
    return rp, ci, row_off, col_off


# ---------------------------------------------------------------- named workloads

WORKLOADS = {
    "er1000": dict(desc="Erdos-Renyi G(n=1000, p=0.02), seed 1"),
    "rmat18": dict(desc="R-MAT scale 18, edge factor 16, a=.57 b=.19 c=.19 d=.05, seed 2"),
    "chunglu1m": dict(desc="Chung-Lu 1M vertices, exponent 2.1, max weight 5000, "
                           "2000 planted cliques of size U[20,60], seed 3"),
    "batch4096": dict(desc="4096 graphs, n log-uniform [50,5000], half ER avg degree U[5,40], "
                           "half planted partition (8 blocks, .3/.005), seed 4"),
    "rmat22": dict(desc="R-MAT scale 22, edge factor 32, a=.57 b=.19 c=.19 d=.05, seed 5"),
}


def cache_dir() -> str:
    return os.environ.get("MCE_GRAPH_CACHE", "/tmp/mce_graph_cache")


def _cached(name: str, make):
    path = os.path.join(cache_dir(), name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return CSRGraph(n=int(z["n"]), row_ptr=z["row_ptr"], col_idx=z["col_idx"], name=name)
    g = make()
    g.name = name
    try:
        os.makedirs(cache_dir(), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, n=np.int64(g.n), row_ptr=g.row_ptr, col_idx=g.col_idx)
        os.replace(tmp, path)
    except OSError:
        pass
    return g


def workload(name: str) -> CSRGraph:
    if name == "er1000":
        return _cached(name, lambda: erdos_renyi(1000, 0.02, 1))
    if name == "rmat18":
        return _cached(name, lambda: rmat(18, 16, 0.57, 0.19, 0.19, 0.05, 2))
    if name == "chunglu1m":
        return _cached(name, lambda: chung_lu_planted(seed=3))
    if name == "rmat22":
        return _cached(name, lambda: rmat(22, 32, 0.57, 0.19, 0.19, 0.05, 5))
    raise KeyError(name)


@dataclass
class Batch:
    """Concatenated CSRs of a batch (the layout of concat_batch)."""

    row_ptr_cat: np.ndarray
    col_idx_cat: np.ndarray
    row_off: np.ndarray
    col_off: np.ndarray

    def __len__(self) -> int:
        return len(self.row_off) - 1

    def graph(self, i: int) -> CSRGraph:
        a, b = int(self.row_off[i]), int(self.row_off[i + 1])
        c, d = int(self.col_off[i]), int(self.col_off[i + 1])
        return CSRGraph(n=b - a - 1, row_ptr=self.row_ptr_cat[a:b], col_idx=self.col_idx_cat[c:d])


def workload_batch(name: str, count: int = 4096, seed: int = 4) -> Batch:
    """Batched workloads, cached like the single graphs: "batch4096" (seed 4)
    and its held-out tuning batch "batch512_tune" (seed 104, 512 graphs)."""
    if name == "batch4096":
        count, seed = 4096, 4
    elif name == "batch512_tune":
        count, seed = 512, 104
    else:
        raise KeyError(name)
    path = os.path.join(cache_dir(), name + ".npz")
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Batch(z["rp"], z["ci"], z["row_off"], z["col_off"])
    rp, ci, row_off, col_off = concat_batch(batch_graphs(count, seed))
    try:
        os.makedirs(cache_dir(), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, rp=rp, ci=ci, row_off=row_off, col_off=col_off)
        os.replace(tmp, path)
    except OSError:
        pass
    return Batch(rp, ci, row_off, col_off)
