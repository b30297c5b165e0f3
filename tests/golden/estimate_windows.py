"""Estimates of how many maximal cliques the core windows beyond the tested
ones hold, by Knuth's tree-size estimator (window_estimate.c) over a
deterministic sample of the roots of each core band.  CPU only; shares
nothing with the library.  Writes tests/golden/window_estimates.json.

usage: python tests/golden/estimate_windows.py [--per-stratum N] [--probes K]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import subprocess
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2212_01473_amd import inputs as I  # noqa: E402
import oracle  # noqa: E402


def load_estimator():
    src = os.path.join(HERE, "window_estimate.c")
    out = os.path.join(ROOT, "oracle", "_build", "libwindow_estimate.so")
    os.makedirs(os.path.dirname(out), exist_ok=True)
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", src, "-o", out])
    lib = C.CDLL(out)
    u32p = C.POINTER(C.c_uint32)
    lib.window_estimate.argtypes = [C.c_uint32, u32p, u32p, u32p, u32p, C.c_uint32, C.c_uint32, C.c_uint64,
                                    C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.window_estimate.restype = C.c_int
    return lib


def band_estimate(lib, g, pos, core, lo, hi, per_stratum, probes, seed):
    """Sum over the roots v with lo <= core(v) <= hi (and a non-empty P) of the
    estimated number of maximal cliques (and tree nodes) below v.  The roots
    are stratified by floor(log2 |P|) (the costs are heavy-tailed in |P|);
    each stratum contributes the mean over an evenly spaced sample of at most
    per_stratum of its roots, times its size."""
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.uint32)
    deg = np.diff(g.row_ptr.astype(np.int64))
    src = np.repeat(np.arange(g.n), deg)
    later = np.bincount(src[pos[g.col_idx.astype(np.int64)] > pos[src]], minlength=g.n)
    band = np.flatnonzero((core >= lo) & (core <= hi) & (later > 0))
    res = dict(lo=int(lo), hi=int(hi), roots=int(band.size), sampled=0, probes=probes, cliques=0.0,
               tree_nodes=0.0, strata=[])
    if band.size == 0:
        return res
    u32p = C.POINTER(C.c_uint32)
    posu = np.ascontiguousarray(pos, dtype=np.uint32)
    t0 = time.time()
    stratum = np.floor(np.log2(later[band])).astype(np.int64)
    for sidx in np.unique(stratum):
        members = band[stratum == sidx]
        step = max(1, -(-members.size // per_stratum))
        sample = np.ascontiguousarray(members[::step].astype(np.uint32))
        est = np.zeros(sample.size)
        nodes = np.zeros(sample.size)
        rc = lib.window_estimate(g.n, rp.ctypes.data_as(u32p), ci.ctypes.data_as(u32p), posu.ctypes.data_as(u32p),
                                 sample.ctypes.data_as(u32p), sample.size, probes, seed,
                                 est.ctypes.data_as(C.POINTER(C.c_double)),
                                 nodes.ctypes.data_as(C.POINTER(C.c_double)))
        if rc != 0:
            raise RuntimeError("a sampled root has more than 4096 later neighbours")
        c, t = float(est.mean() * members.size), float(nodes.mean() * members.size)
        res["cliques"] += c
        res["tree_nodes"] += t
        res["sampled"] += int(sample.size)
        res["strata"].append(dict(p_from=int(2 ** sidx), roots=int(members.size), sampled=int(sample.size),
                                  cliques=c, tree_nodes=t))
    res["seconds"] = round(time.time() - t0, 1)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--per-stratum", type=int, default=200)
    ap.add_argument("--probes", type=int, default=1024, help="walks per sampled root, tested window and next band")
    ap.add_argument("--probes-far", type=int, default=32, help="walks per sampled root, the bands beyond")
    args = ap.parse_args()
    lib = load_estimator()
    out = {"method": "Knuth (1975) tree-size estimator below each sampled root; order of magnitude only",
           "per_stratum": args.per_stratum, "workloads": {}}
    # the first band of each is the tested window itself (known totals: R-MAT 18
    # c = 264 holds 41,848,495 maximal cliques, R-MAT 22 c = 425 holds
    # 2,510,844,632), a check of the estimator's scale
    plans = {"rmat18": [(0, 264), (265, 265), (266, 300), (301, 370)],
             "rmat22": [(0, 425), (426, 426), (427, 512), (513, 1024), (1025, 1687)]}
    for name, bands in plans.items():
        g = I.workload(name)
        order, rank = oracle.sync_order(g)
        core, _, _ = oracle.sync_peel(g)
        pos = rank.astype(np.int64)
        res = []
        for i, (lo, hi) in enumerate(bands):
            probes = args.probes if i < 2 else args.probes_far
            r = band_estimate(lib, g, pos, core, lo, hi, args.per_stratum, probes, seed=12345)
            print(name, {k: v for k, v in r.items() if k != "strata"}, flush=True)
            res.append(r)
        out["workloads"][name] = res
    with open(os.path.join(HERE, "window_estimates.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
