"""Write the stored oracle results of the full-size workloads.

Calls only the oracle (oracle/) and the seeded input generators; nothing here
touches the HIP library.  Each entry records the SHA-256 of the generated CSR,
so a test can check it enumerates the same graph.

tests/golden/workloads.json:
  rmat18_c264       R-MAT scale 18 (ef 16, seed 2), core window 264: count, hash, histogram
  chunglu1m         Chung-Lu 1M + 2000 planted cliques (seed 3), full: count, hash, histogram
  batch4096_sample  every 64th graph of the 4096-graph batch (seed 4): per-graph results
  rmat22_c425_roots R-MAT scale 22 (ef 32, seed 5), window 425, roots with input id
                    divisible by 16384, attributed in the synchronous-peel order (the
                    order the library uses): count and hash of the cliques they report
  rmat22_c425       the whole R-MAT 22 window c = 425: count, hash, histogram.  Run in
                    64 parts (roots v with v % 64 == j, each in the oracle's own bucket
                    order); the parts' sums are the window's results because every
                    maximal clique is reported by exactly one root (Algorithm 3)

tests/golden/batch4096_full.json:
  every one of the 4096 graphs of the batch: count, hash and histogram per graph,
  the SHA-256 of the concatenated batch arrays, and per-graph SHA-256 prefixes

Run: python tests/golden/make_workload_golden.py [entry ...] [--threads T] [--partial DIR]
(hours on 8 cores for rmat22_c425 and batch4096_full; the partial results of
the long entries are kept in DIR, default /tmp, so an interrupted run resumes)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2212_01473_amd import inputs as I  # noqa: E402

OUT = os.path.join(HERE, "workloads.json")
OUT_BATCH = os.path.join(HERE, "batch4096_full.json")
BATCH_EVERY = 64
RMAT22_ROOT_MOD = 16384
RMAT22_PARTS = 64
MASK64 = (1 << 64) - 1


def hist_dict(h):
    return {str(k): int(v) for k, v in enumerate(h) if v}


def full(g, c, threads=0):
    t0 = time.time()
    r = oracle.mce(g, max_root_core=c, threads=threads)
    return {"sha256": g.sha256(), "window": int(c), "count": int(r.count), "hash": f"{int(r.hash):#018x}",
            "hist": hist_dict(r.hist), "oracle_seconds": round(time.time() - t0, 1), "threads": int(r.threads)}


def _load_partial(path):
    return json.load(open(path)) if os.path.exists(path) else {}


def _save_partial(path, data):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f)
    os.replace(tmp, path)


def rmat22_window(threads, partial_dir):
    g = I.workload("rmat22")
    sha = g.sha256()
    path = os.path.join(partial_dir, f"mce_golden_rmat22_c425_{sha[:16]}.json")
    parts = _load_partial(path)
    ids = np.arange(g.n)
    for j in range(RMAT22_PARTS):
        if str(j) in parts:
            continue
        t0 = time.time()
        mask = (ids % RMAT22_PARTS == j).astype(np.uint8)
        r = oracle.mce(g, max_root_core=425, root_mask=mask, threads=threads)
        parts[str(j)] = {"count": int(r.count), "hash": int(r.hash), "hist": [int(x) for x in r.hist],
                         "seconds": round(time.time() - t0, 1), "threads": int(r.threads)}
        _save_partial(path, parts)
        print(f"rmat22_c425 part {j}: {r.count} cliques in {time.time() - t0:.1f}s", flush=True)
    count, h, hist = 0, 0, {}
    for p in parts.values():
        count += p["count"]
        h = (h + p["hash"]) & MASK64
        for k, v in enumerate(p["hist"]):
            if v:
                hist[str(k)] = hist.get(str(k), 0) + v
    return {"sha256": sha, "window": 425, "parts": RMAT22_PARTS, "count": count, "hash": f"{h:#018x}",
            "hist": dict(sorted(hist.items(), key=lambda kv: int(kv[0]))),
            "oracle_seconds": round(sum(p["seconds"] for p in parts.values()), 1),
            "threads": max(p["threads"] for p in parts.values())}


def batch_sha256(batch) -> str:
    h = hashlib.sha256()
    for a in (batch.row_ptr_cat, batch.col_idx_cat, batch.row_off, batch.col_off):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def batch_full(threads, partial_dir):
    batch = I.workload_batch("batch4096")
    sha = batch_sha256(batch)
    path = os.path.join(partial_dir, f"mce_golden_batch4096_{sha[:16]}.json")
    done = _load_partial(path)
    t_last = time.time()
    for i in range(len(batch)):
        if str(i) in done:
            continue
        g = batch.graph(i)
        t0 = time.time()
        r = oracle.mce(g, threads=threads)
        done[str(i)] = [int(r.count), f"{int(r.hash):#018x}", hist_dict(r.hist), g.sha256()[:16],
                        round(time.time() - t0, 2)]
        if time.time() - t_last > 30 or i == len(batch) - 1:
            _save_partial(path, done)
            t_last = time.time()
            print(f"batch4096_full: {len(done)} of {len(batch)} graphs", flush=True)
    _save_partial(path, done)
    graphs = [done[str(i)] for i in range(len(batch))]
    return {"batch_sha256": sha, "n_graphs": len(batch),
            "oracle_seconds": round(sum(x[4] for x in graphs), 1),
            "fields": ["count", "hash", "hist", "graph_sha256_prefix"],
            "graphs": [x[:4] for x in graphs]}


def make(name, threads, partial_dir):
    if name == "rmat18_c264":
        return full(I.workload("rmat18"), 264, threads)
    if name == "chunglu1m":
        return full(I.workload("chunglu1m"), 0xFFFFFFFF, threads)
    if name == "batch4096_sample":
        batch = I.workload_batch("batch4096")
        graphs = {}
        t0 = time.time()
        for i in range(0, len(batch), BATCH_EVERY):
            g = batch.graph(i)
            r = oracle.mce(g, threads=threads)
            graphs[str(i)] = {"sha256": g.sha256(), "count": int(r.count), "hash": f"{int(r.hash):#018x}",
                              "hist": hist_dict(r.hist)}
        return {"every": BATCH_EVERY, "graphs": graphs, "oracle_seconds": round(time.time() - t0, 1)}
    if name == "rmat22_c425_roots":
        g = I.workload("rmat22")
        order, _ = oracle.sync_order(g)
        mask = (np.arange(g.n) % RMAT22_ROOT_MOD == 0).astype(np.uint8)
        t0 = time.time()
        r = oracle.mce(g, max_root_core=425, root_mask=mask, order=order, threads=threads)
        return {"sha256": g.sha256(), "window": 425, "root_mod": RMAT22_ROOT_MOD, "n_roots": int(mask.sum()),
                "count": int(r.count), "hash": f"{int(r.hash):#018x}", "oracle_seconds": round(time.time() - t0, 1)}
    if name == "rmat22_c425":
        return rmat22_window(threads, partial_dir)
    if name == "batch4096_full":
        return batch_full(threads, partial_dir)
    raise KeyError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--partial", default="/tmp")
    args = ap.parse_args()
    names = args.names or ["rmat18_c264", "chunglu1m", "batch4096_sample", "rmat22_c425_roots",
                           "rmat22_c425", "batch4096_full"]
    for name in names:
        t0 = time.time()
        entry = make(name, args.threads, args.partial)
        out = OUT_BATCH if name == "batch4096_full" else OUT
        data = json.load(open(out)) if (out == OUT and os.path.exists(out)) else {}
        if out == OUT_BATCH:
            data = entry
        else:
            data[name] = entry
        with open(out, "w") as f:
            json.dump(data, f, indent=None if out == OUT_BATCH else 1, sort_keys=out == OUT,
                      separators=(",", ":") if out == OUT_BATCH else None)
        print(f"{name}: done in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main()
