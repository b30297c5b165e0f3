"""The core-window estimator (tests/golden/window_estimate.c, Knuth's
tree-size estimator below first-level roots) against exact counts."""
import ctypes as C
import os
import sys

import numpy as np

import oracle
from paper_2212_01473_amd import inputs as I

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import estimate_windows as EW  # noqa: E402


def _estimate(g, probes):
    lib = EW.load_estimator()
    _, rank = oracle.sync_order(g)
    roots = np.arange(g.n, dtype=np.uint32)
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.uint32)
    pos = np.ascontiguousarray(rank, dtype=np.uint32)
    est = np.zeros(g.n)
    nodes = np.zeros(g.n)
    u32p = C.POINTER(C.c_uint32)
    rc = lib.window_estimate(g.n, rp.ctypes.data_as(u32p), ci.ctypes.data_as(u32p), pos.ctypes.data_as(u32p),
                             roots.ctypes.data_as(u32p), g.n, probes, 7, est.ctypes.data_as(C.POINTER(C.c_double)),
                             nodes.ctypes.data_as(C.POINTER(C.c_double)))
    assert rc == 0
    return est, nodes


def test_uniform_tree_is_estimated_exactly():
    # Moon-Moser with k parts of 3: every search path below a root branches
    # the same way, so each single walk gives the exact clique count
    g = I.moon_moser(4)
    est, _ = _estimate(g, 1)
    assert round(est.sum(), 9) == oracle.mce(g).count == 81


def test_estimate_converges_to_the_count():
    # unbiased: the mean over many walks approaches the oracle's count
    g = I.erdos_renyi(60, 0.3, 11)
    exact = oracle.mce(g).count
    est, nodes = _estimate(g, 20000)
    assert abs(est.sum() - exact) <= 0.05 * exact, (est.sum(), exact)
    assert nodes.sum() >= est.sum()
