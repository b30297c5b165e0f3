"""Write tests/golden/workloads.json: oracle results on the full-size workloads.

Calls only the oracle (oracle/) and the seeded input generators; nothing here
touches the HIP library.  Each entry records the SHA-256 of the generated CSR,
so a test can check it enumerates the same graph.  Entries:

  rmat18_c264       R-MAT scale 18 (ef 16, seed 2), core window 264: count, hash, histogram
  chunglu1m         Chung-Lu 1M + 2000 planted cliques (seed 3), full: count, hash, histogram
  batch4096_sample  every 64th graph of the 4096-graph batch (seed 4): per-graph results
  rmat22_c425_roots R-MAT scale 22 (ef 32, seed 5), window 425, roots with input id
                    divisible by 16384, attributed in the synchronous-peel order (the
                    order the library uses): count and hash of the cliques they report

Run: python tests/golden/make_workload_golden.py [entry ...]   (minutes on 8 cores)
"""
from __future__ import annotations

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
BATCH_EVERY = 64
RMAT22_ROOT_MOD = 16384


def hist_dict(h):
    return {str(k): int(v) for k, v in enumerate(h) if v}


def full(g, c):
    t0 = time.time()
    r = oracle.mce(g, max_root_core=c)
    return {"sha256": g.sha256(), "window": int(c), "count": int(r.count), "hash": f"{int(r.hash):#018x}",
            "hist": hist_dict(r.hist), "oracle_seconds": round(time.time() - t0, 1), "threads": int(r.threads)}


def make(name):
    if name == "rmat18_c264":
        return full(I.workload("rmat18"), 264)
    if name == "chunglu1m":
        return full(I.workload("chunglu1m"), 0xFFFFFFFF)
    if name == "batch4096_sample":
        batch = I.workload_batch("batch4096")
        graphs = {}
        t0 = time.time()
        for i in range(0, len(batch), BATCH_EVERY):
            g = batch.graph(i)
            r = oracle.mce(g)
            graphs[str(i)] = {"sha256": g.sha256(), "count": int(r.count), "hash": f"{int(r.hash):#018x}",
                              "hist": hist_dict(r.hist)}
        return {"every": BATCH_EVERY, "graphs": graphs, "oracle_seconds": round(time.time() - t0, 1)}
    if name == "rmat22_c425_roots":
        g = I.workload("rmat22")
        order, _ = oracle.sync_order(g)
        mask = (np.arange(g.n) % RMAT22_ROOT_MOD == 0).astype(np.uint8)
        t0 = time.time()
        r = oracle.mce(g, max_root_core=425, root_mask=mask, order=order)
        return {"sha256": g.sha256(), "window": 425, "root_mod": RMAT22_ROOT_MOD, "n_roots": int(mask.sum()),
                "count": int(r.count), "hash": f"{int(r.hash):#018x}", "oracle_seconds": round(time.time() - t0, 1)}
    raise KeyError(name)


def main():
    names = sys.argv[1:] or ["rmat18_c264", "chunglu1m", "batch4096_sample", "rmat22_c425_roots"]
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        t0 = time.time()
        data[name] = make(name)
        print(f"{name}: done in {time.time() - t0:.1f}s", flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
