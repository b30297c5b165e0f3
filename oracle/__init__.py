"""CPU oracle for maximal clique enumeration -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it, and it imports nothing from there.

Contents:

* ``mce(graph, ...)``: Algorithm 3 (independent first-level subtrees over a
  degeneracy order) calling Algorithm 2 (Bron-Kerbosch with Tomita pivoting),
  in plain C (``mce_oracle.c``), with an optional core window.
* ``degeneracy`` / ``sync_peel``: degeneracy order and core numbers, and the
  sequential simulation of the synchronous-round peel whose arrays the GPU
  peel must reproduce exactly.
* ``clique_hash`` / ``key``: the clique hash, defined from SplitMix64.
* ``brute_force``: subset enumeration straight from the definition of a
  maximal clique (Section II-A), for graphs of at most 20 vertices.
* ``bk_no_pivot``: Algorithm 1 (plain Bron-Kerbosch over the whole vertex set)
  in pure Python, for tiny graphs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libmce_oracle.so")
_SRC = os.path.join(_HERE, "mce_oracle.c")
_lib = None

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Result(C.Structure):
    _fields_ = [("count", C.c_uint64), ("hash", C.c_uint64), ("nodes", C.c_uint64),
                ("cliques_written", C.c_uint64), ("verts_written", C.c_uint64),
                ("max_size", C.c_uint32), ("degeneracy", C.c_uint32),
                ("status", C.c_int32), ("threads", C.c_int32)]


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_LIB_PATH)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        lib.oracle_key.restype = C.c_uint64
        lib.oracle_key.argtypes = [C.c_uint64]
        lib.oracle_clique_hash.restype = C.c_uint64
        lib.oracle_clique_hash.argtypes = [u32p, C.c_uint32]
        lib.oracle_degeneracy.restype = C.c_int
        lib.oracle_degeneracy.argtypes = [C.c_uint32, u32p, u32p, u32p, u32p]
        lib.oracle_sync_peel.restype = C.c_int64
        lib.oracle_sync_peel.argtypes = [C.c_uint32, u32p, u32p, u32p, u32p]
        lib.oracle_mce.restype = C.c_int
        lib.oracle_mce.argtypes = [C.c_uint32, u32p, u32p, C.c_uint32, C.c_int,
                                   u64p, C.c_uint32, u32p, C.c_uint64, u64p, C.c_uint64,
                                   C.POINTER(C.c_uint8), C.POINTER(C.c_uint32), C.POINTER(_Result)]
        lib.oracle_max_threads.restype = C.c_int
        _lib = lib
    return _lib


def _u32(a):
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint32))


def key(v: int) -> int:
    return int(_load().oracle_key(v))


def clique_hash(ids) -> int:
    a, p = _u32(np.asarray(list(ids), dtype=np.uint32))
    return int(_load().oracle_clique_hash(p, len(a)))


@dataclass
class MCEResult:
    count: int
    hash: int
    hist: np.ndarray
    max_size: int
    degeneracy: int
    nodes: int
    threads: int
    cliques: list | None = field(default=None)


def mce(g, max_root_core: int = 0xFFFFFFFF, threads: int = 0, collect: bool = False,
        root_mask: np.ndarray | None = None, order: np.ndarray | None = None) -> MCEResult:
    """Exact maximal cliques of ``g`` (a CSR graph) with min core <= max_root_core.
    ``order`` (a core-sorted permutation) replaces the bucket degeneracy order;
    it changes which root reports a clique, never the set of cliques."""
    lib = _load()
    rp, rpp = _u32(g.row_ptr)
    ci, cip = _u32(g.col_idx)
    n = int(g.n)
    hist_len = 4096
    hist = np.zeros(hist_len, dtype=np.uint64)
    res = _Result()
    vp = op = None
    verts = offs = None
    vcap = ocap = 0
    if collect:
        vcap = 1 << 22
        ocap = 1 << 20
        verts = np.zeros(vcap, dtype=np.uint32)
        offs = np.zeros(ocap, dtype=np.uint64)
        vp = verts.ctypes.data_as(C.POINTER(C.c_uint32))
        op = offs.ctypes.data_as(C.POINTER(C.c_uint64))
    mask_p = None
    if root_mask is not None:
        mask = np.ascontiguousarray(root_mask, dtype=np.uint8)
        mask_p = mask.ctypes.data_as(C.POINTER(C.c_uint8))
    order_p = None
    if order is not None:
        order_a = np.ascontiguousarray(order, dtype=np.uint32)
        assert order_a.shape[0] == n
        order_p = order_a.ctypes.data_as(C.POINTER(C.c_uint32))
    st = lib.oracle_mce(n, rpp, cip, int(max_root_core) & 0xFFFFFFFF, int(threads),
                        hist.ctypes.data_as(C.POINTER(C.c_uint64)), hist_len,
                        vp, vcap, op, ocap, mask_p, order_p, C.byref(res))
    if st < 0:
        raise MemoryError("oracle ran out of memory")
    if st == 1:
        raise RuntimeError("oracle clique buffer overflow")
    cliques = None
    if collect:
        cliques = []
        prev = 0
        for i in range(int(res.cliques_written)):
            end = int(offs[i])
            cliques.append(tuple(sorted(int(x) for x in verts[prev:end])))
            prev = end
    top = int(res.max_size)
    return MCEResult(count=int(res.count), hash=int(res.hash), hist=hist[: top + 1].copy(),
                     max_size=top, degeneracy=int(res.degeneracy), nodes=int(res.nodes),
                     threads=int(res.threads), cliques=cliques)


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def degeneracy(g):
    """(order, core) by the Batagelj-Zaversnik bucket algorithm."""
    lib = _load()
    rp, rpp = _u32(g.row_ptr)
    ci, cip = _u32(g.col_idx)
    order = np.zeros(max(g.n, 1), dtype=np.uint32)
    core = np.zeros(max(g.n, 1), dtype=np.uint32)
    lib.oracle_degeneracy(g.n, rpp, cip, order.ctypes.data_as(C.POINTER(C.c_uint32)),
                          core.ctypes.data_as(C.POINTER(C.c_uint32)))
    return order[: g.n], core[: g.n]


def sync_peel(g):
    """(core, round, n_rounds) of the synchronous-round peel."""
    lib = _load()
    rp, rpp = _u32(g.row_ptr)
    ci, cip = _u32(g.col_idx)
    core = np.zeros(max(g.n, 1), dtype=np.uint32)
    rnd = np.zeros(max(g.n, 1), dtype=np.uint32)
    r = lib.oracle_sync_peel(g.n, rpp, cip, core.ctypes.data_as(C.POINTER(C.c_uint32)),
                             rnd.ctypes.data_as(C.POINTER(C.c_uint32)))
    return core[: g.n], rnd[: g.n], int(r)


def sync_order(g):
    """The order sorted by (core, round, id) of the synchronous peel, and the
    rank of every vertex in it."""
    core, rnd, _ = sync_peel(g)
    order = np.lexsort((np.arange(g.n), rnd, core)).astype(np.uint32)
    rank = np.empty(g.n, dtype=np.uint32)
    rank[order] = np.arange(g.n, dtype=np.uint32)
    return order, rank


# ------------------------------------------------------------------ pure-Python references

def adjacency_masks(g) -> list[int]:
    masks = []
    for v in range(g.n):
        m = 0
        for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]:
            m |= 1 << int(u)
        masks.append(m)
    return masks


def brute_force(g):
    """All maximal cliques straight from the definition (Section II-A): every
    non-empty vertex subset that is pairwise adjacent and to which no further
    vertex can be added.  Vectorised over all 2^n subsets; n <= 20."""
    n = g.n
    if n > 20:
        raise ValueError("brute force limited to n <= 20")
    if n == 0:
        return []
    adj = adjacency_masks(g)
    S = np.arange(1 << n, dtype=np.int64)
    clique = S != 0
    for i in range(n):
        has_i = (S >> i) & 1 == 1
        others = S & ~(1 << i)
        clique &= ~has_i | ((others & ~adj[i]) == 0)
    extendable = np.zeros_like(clique)
    for j in range(n):
        not_in = (S >> j) & 1 == 0
        extendable |= not_in & ((S & ~adj[j]) == 0)
    maximal = np.flatnonzero(clique & ~extendable)
    return [tuple(i for i in range(n) if (int(s) >> i) & 1) for s in maximal]


def bk_no_pivot(g):
    """Algorithm 1: plain Bron-Kerbosch with R empty, P = V, X empty."""
    nbr = [set(int(u) for u in g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]) for v in range(g.n)]
    out = []

    def rec(R, P, X):
        if not P and not X:
            if R:
                out.append(tuple(sorted(R)))
            return
        for v in sorted(P):
            rec(R | {v}, P & nbr[v], X & nbr[v])
            P = P - {v}
            X = X | {v}

    rec(set(), set(range(g.n)), set())
    return out


def summarize(cliques):
    """(count, hist, hash) of an explicit list of cliques."""
    hist = {}
    h = 0
    for c in cliques:
        hist[len(c)] = hist.get(len(c), 0) + 1
        h = (h + clique_hash(c)) & MASK64
    top = max(hist) if hist else 0
    arr = np.zeros(top + 1, dtype=np.uint64)
    for k, v in hist.items():
        arr[k] = v
    return len(cliques), arr, h
