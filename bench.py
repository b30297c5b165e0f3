"""Benchmark: exact maximal clique enumeration on one MI355X.

One step = the whole hot path over input already resident in HBM: device
validation of the CSR, the synchronous-round peel and degeneracy order,
orientation into later/earlier neighbour lists, the root queue (for the
learned form: root features, BF16 cost-model inference, ordering and split),
and the persistent enumeration kernel, ending with the results on the host.

Workloads (seeded synthetic graphs shaped like the paper's inputs):
  rmat22     R-MAT scale 22, edge factor 32, a=.57 b=.19 c=.19 d=.05, seed 5,
             core window c = 425 (default: the largest single-GPU workload)
  rmat18     R-MAT scale 18, edge factor 16, same quadrants, seed 2, window c = 264
  chunglu1m  Chung-Lu 1M vertices (exponent 2.1, max weight 5000) + 2000 planted
             cliques of size U[20,60], seed 3, full enumeration
  er1000     Erdos-Renyi G(1000, 0.02), seed 1, full enumeration
  batch4096  4096 graphs (n log-uniform [50, 5000]; half Erdos-Renyi with average
             degree U[5,40], half planted partition 8 blocks .3/.005), seed 4

Forms:
  plain      degeneracy-order root queue, worker list, default knobs
  learned    roots ordered by the cost model (trained beforehand on scale-18
             R-MAT graphs of other seeds, outside the timed region) and the
             costliest split into groups of level-1 branches
  batched    (batch4096) every graph in one launch, knobs autotuned beforehand
             on a held-out batch (512 graphs, seed 104)
  batched_learned  the batched form with the learned order and split
  sequential (batch4096) one load + enumerate per graph, plain form

By default the line reports R-MAT 22 in the learned form with the plain form
timed beside it at equal results, and a "batch" section with the 4096-graph
batch in the batched+learned, batched and sequential forms.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FULL = 0xFFFFFFFF
WORKLOADS = {
    "er1000": dict(kind="graph", c=FULL, form="plain", compare="", cpu_mod=1,
                   desc="Erdos-Renyi G(n=1000, p=0.02), seed 1, full enumeration"),
    "rmat18": dict(kind="graph", c=264, form="plain", compare="learned", cpu_mod=4,
                   desc="R-MAT scale 18, edge factor 16, a=.57 b=.19 c=.19 d=.05, seed 2, core window c=264"),
    "chunglu1m": dict(kind="graph", c=FULL, form="plain", compare="learned", cpu_mod=4,
                      desc="Chung-Lu 1M vertices, exponent 2.1, max weight 5000, 2000 planted cliques U[20,60], "
                           "seed 3, full enumeration"),
    "rmat22": dict(kind="graph", c=425, form="learned", compare="plain", cpu_mod=256,
                   desc="R-MAT scale 22, edge factor 32, a=.57 b=.19 c=.19 d=.05, seed 5, core window c=425"),
    "batch4096": dict(kind="batch", c=FULL, form="batched_learned", compare="batched,sequential", cpu_mod=64,
                      desc="4096 graphs, n log-uniform [50,5000], half ER avg degree U[5,40], half planted "
                           "partition (8 blocks, p_in .3, p_out .005), seed 4, full enumeration"),
}

# MI355X peaks (published; gfx950 unit counts at the 2.4 GHz peak clock)
HBM_PEAK_GBS = 8000.0
CUS, SIMDS, CLOCK_GHZ = 256, 4, 2.4
# one wave64 VALU instruction per SIMD every 4 cycles; one scalar instruction per CU and cycle
VALU_PEAK_GINST = CUS * SIMDS * CLOCK_GHZ / 4
SALU_PEAK_GINST = CUS * CLOCK_GHZ
# LDS: 128 bytes per CU and cycle
LDS_PEAK_GBS = CUS * 128 * CLOCK_GHZ


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# Algorithmic HBM bytes of one enumeration launch, from the kernel's own counters:
#   4 B per adjacency entry scanned to build bitmap rows,
#   8 B per P/X id staged from the oriented CSR for a root (read + write),
#   12 B per X_X adjacency test on the index list (the id and two row pointers),
#   8 B per X-column word read for a bitmap X_X,
#   4 B per list entry probed by the binary searches of those tests.
def algorithmic_bytes(stats) -> int:
    return (4 * stats["build_edges"] + 8 * stats["root_words"] + 12 * stats["xtests"]
            + 8 * stats["xcol_words"] + 4 * stats["probes"])


def kernel_source_sha() -> str:
    src = os.path.join(ROOT, "paper_2212_01473_amd", "csrc", "enumerate.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def committed_profile(kind: str, workload: str, c: int):
    """A committed rocprofv3 counter summary of k_enumerate (profiles/*_<kind>.json)
    taken on the current kernel source and on this workload, else None."""
    sha = kernel_source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", f"k_enumerate_*_{kind}.json"))):
        d = json.load(open(path))
        if d.get("source_sha256_prefix") == sha and d.get("workload") == f"{workload} c={c}":
            d["file"] = os.path.relpath(path, ROOT)
            return d
    return None


def rooflines(workload: str, c: int, st, kern_ms: float):
    """The roofline objects of the dominant kernel (k_enumerate).  Instruction
    issue binds it: the SQ counter summary gives instructions per tree node,
    scaled to this launch's nodes and divided by the live kernel time.  HBM:
    the kernel's algorithmic bytes over the same time; traffic from the
    FETCH_SIZE / WRITE_SIZE summary.  LDS: the bytes of the LDS instructions
    counted, at most 8 bytes per lane."""
    sec = kern_ms / 1e3
    alg = algorithmic_bytes(st)
    traffic = committed_profile("traffic", workload, c)
    hbm = {"bound": "hbm", "kernel": "k_enumerate", "achieved": round(alg / sec / 1e9, 2), "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": round(alg / sec / 1e9 / HBM_PEAK_GBS, 5),
           "traffic": (traffic["fetch_bytes"] + traffic["write_bytes"]) if traffic else None,
           "algorithmic_bytes": alg, "avg_kernel_ms": round(kern_ms, 3)}
    sq = committed_profile("sq", workload, c)
    if sq is None:
        return hbm, {"hbm": hbm}
    nodes = st["nodes"]
    valu = sq["valu_per_node"] * nodes / sec / 1e9
    salu = sq["salu_per_node"] * nodes / sec / 1e9
    lds = sq["lds_per_node"] * nodes * 64 * 8 / sec / 1e9
    fv, fs = valu / VALU_PEAK_GINST, salu / SALU_PEAK_GINST
    issue = {"bound": "alu", "kernel": "k_enumerate", "achieved": round(max(valu, salu), 2),
             "peak": round(VALU_PEAK_GINST if fv >= fs else SALU_PEAK_GINST, 1), "unit": "Ginst/s",
             "frac": round(max(fv, fs), 4), "traffic": hbm["traffic"],
             "binding": "valu issue" if fv >= fs else "salu issue",
             "valu": {"achieved": round(valu, 2), "peak": round(VALU_PEAK_GINST, 1), "frac": round(fv, 4)},
             "salu": {"achieved": round(salu, 2), "peak": round(SALU_PEAK_GINST, 1), "frac": round(fs, 4)},
             "per_node": {k: sq[k] for k in ("valu_per_node", "salu_per_node", "lds_per_node", "vmem_per_node")},
             "counters": sq["file"], "avg_kernel_ms": round(kern_ms, 3)}
    lds_o = {"bound": "lds", "achieved": round(lds, 2), "peak": round(LDS_PEAK_GBS, 1), "unit": "GB/s",
             "frac": round(lds / LDS_PEAK_GBS, 5), "note": "upper bound: 8 bytes per lane of every LDS instruction"}
    return issue, {"hbm": hbm, "lds": lds_o}


def cpu_baseline_graph(g, c, frac_mod: int):
    """The oracle as it stands, on a deterministic sample of roots (input ids
    v with v % frac_mod == 0) with all host threads it is given, and on a
    sample 16 times smaller with one thread."""
    import oracle

    mask = (np.arange(g.n) % frac_mod == 0).astype(np.uint8)
    t0 = time.perf_counter()
    r = oracle.mce(g, max_root_core=c, root_mask=mask)
    dt = time.perf_counter() - t0
    mask1 = (np.arange(g.n) % (16 * frac_mod) == 0).astype(np.uint8)
    t1 = time.perf_counter()
    r1 = oracle.mce(g, max_root_core=c, root_mask=mask1, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": r.count / dt, "unit": "cliques/s", "cores": int(r.threads), "kind": "oracle",
            "sample": f"roots with input id % {frac_mod} == 0 ({int(mask.sum())} of {g.n}); "
                      f"{r.count} cliques in {dt:.2f} s", "seconds": round(dt, 3),
            "single_thread": {"value": r1.count / dt1, "cores": 1,
                              "sample": f"roots with input id % {16 * frac_mod} == 0; {r1.count} cliques in "
                                        f"{dt1:.2f} s"}}


def cpu_baseline_batch(batch, every: int):
    """The oracle on every `every`-th graph of the batch."""
    import oracle

    idx = list(range(0, len(batch), every))
    t0 = time.perf_counter()
    count, threads = 0, 1
    for i in idx:
        r = oracle.mce(batch.graph(i))
        count += r.count
        threads = r.threads
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "cliques/s", "cores": int(threads), "kind": "oracle",
            "sample": f"graphs with index % {every} == 0 ({len(idx)} of {len(batch)}); {count} cliques in "
                      f"{dt:.2f} s", "seconds": round(dt, 3)}


def timed(steps, f, nsteps, nwarm):
    """nwarm untimed steps, then nsteps timed between device synchronisations;
    every step must give the same results."""
    import torch

    for i in range(nwarm):
        res, st, _ = steps[f]()
        log(f"[bench] {f} warmup {i}: count={sum(r.count for r in res)} kernel={st['kernel_ns'] / 1e6:.1f}ms")
    torch.cuda.synchronize()
    out = []
    t0 = time.perf_counter()
    for _ in range(nsteps):
        out.append(steps[f]())
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    keys = {tuple((r.count, r.hash) for r in res) for res, _, _ in out}
    assert len(keys) == 1, f"{f}: results differ between steps"
    return out, el / nsteps


def result_key(res):
    return tuple((r.count, r.hash, tuple(r.hist.tolist())) for r in res)


def graph_steps(name, c, knobs, forms, load_kw=None):
    """Step callables of a single-graph workload for the requested forms."""
    import torch

    from paper_2212_01473_amd import inputs as I
    from paper_2212_01473_amd import mce

    t0 = time.perf_counter()
    g = I.workload(name)
    log(f"[bench] workload {name}: n={g.n} m={g.m} ready in {time.perf_counter() - t0:.1f}s")
    rp = torch.from_numpy(g.row_ptr.astype(np.int64)).to(torch.int32).cuda()
    ci = torch.from_numpy(g.col_idx.astype(np.int64)).to(torch.int32).cuda()
    model = None
    if "learned" in forms:
        from paper_2212_01473_amd import learned

        t1 = time.perf_counter()
        model = learned.cached_model()
        log(f"[bench] cost model ready in {time.perf_counter() - t1:.1f}s")

    def graph_step(extra):
        def step():
            dg = mce.load_csr(rp, ci, g.n, **(load_kw or {}))
            info = dg.info()
            r = mce.enumerate_cliques(dg, max_root_core=c, hist_len=info.degeneracy + 2, **knobs, **extra)
            dg.free()
            return [r], r.stats, info
        return step

    steps = {"plain": graph_step({}), "l2": graph_step(dict(l2_roots=True))}
    if model is not None:
        steps["learned"] = graph_step(dict(model=model, split=True))
    return g, steps


def batch_steps(knobs, forms):
    import torch

    from paper_2212_01473_amd import inputs as I
    from paper_2212_01473_amd import mce

    t0 = time.perf_counter()
    batch = I.workload_batch("batch4096")
    log(f"[bench] batch4096: {len(batch)} graphs, {int(batch.row_off[-1]) - len(batch)} vertices, "
        f"{batch.col_idx_cat.size // 2} edges, ready in {time.perf_counter() - t0:.1f}s")
    rp = torch.from_numpy(batch.row_ptr_cat.astype(np.int64)).to(torch.int32).cuda()
    ci = torch.from_numpy(batch.col_idx_cat.astype(np.int64)).to(torch.int32).cuda()
    # knobs tuned on a held-out batch, outside the timed region
    t1 = time.perf_counter()
    tb = I.workload_batch("batch512_tune")
    trp = torch.from_numpy(tb.row_ptr_cat.astype(np.int64)).to(torch.int32).cuda()
    tci = torch.from_numpy(tb.col_idx_cat.astype(np.int64)).to(torch.int32).cuda()
    with mce.load_batch_device(trp, tci, tb.row_off, tb.col_off) as tg:
        tuned, rep = mce.autotune(tg, **knobs)
    log(f"[bench] autotuned on the held-out batch in {time.perf_counter() - t1:.1f}s: {rep}")
    del trp, tci
    bmodel = None
    if "batched_learned" in forms:
        from paper_2212_01473_amd import learned

        bmodel = learned.cached_model()

    def batched():
        dg = mce.load_batch_device(rp, ci, batch.row_off, batch.col_off)
        res = mce.enumerate_batch(dg, options=tuned)
        dg.free()
        return res, res[0].stats, None

    def batched_learned():
        dg = mce.load_batch_device(rp, ci, batch.row_off, batch.col_off)
        opt = mce.make_options(**knobs, model=bmodel, split=True)
        for k in ("donate_min_p", "bitmap_max_p", "wg_per_cu", "donate_max_depth", "xrow_ratio"):
            setattr(opt, k, getattr(tuned, k))
        res = mce.enumerate_batch(dg, options=opt)
        dg.free()
        return res, res[0].stats, None

    def sequential():
        res, stats = [], None
        for i in range(len(batch)):
            a, b = int(batch.row_off[i]), int(batch.row_off[i + 1])
            cc, d = int(batch.col_off[i]), int(batch.col_off[i + 1])
            dg = mce.load_csr(rp[a:b], ci[cc:d] if d > cc else ci[:1], b - a - 1)
            r = mce.enumerate_cliques(dg, **knobs)
            dg.free()
            res.append(r)
            stats = r.stats
        return res, stats, None

    steps = {"batched": batched, "batched_learned": batched_learned, "sequential": sequential}
    return batch, steps, rep


def compare_forms(steps, forms, key, nsteps, nwarm, reported_sec, count):
    comp = {}
    for f in forms:
        one = f == "sequential"
        cr, csec = timed(steps, f, 1 if one else nsteps, 0 if one else nwarm)
        assert result_key(cr[-1][0]) == key, f"form {f} changed the results"
        comp[f] = {"ms_per_step": round(csec * 1e3, 3), "value": count / csec,
                   "kernel_ms": round(cr[-1][1]["kernel_ns"] / 1e6, 3),
                   "setup_ms": round(cr[-1][1]["setup_ns"] / 1e6, 3),
                   "reported_form_speedup": round(csec / reported_sec, 3)}
        log(f"[bench] {f}: {csec * 1e3:.1f} ms/step (reported form: {reported_sec * 1e3:.1f})")
    return comp


def batch_section(args, knobs):
    """The 4096-graph batch: batched+learned (reported), batched, sequential."""
    spec = WORKLOADS["batch4096"]
    forms = ["batched_learned", "batched", "sequential"]
    batch, steps, rep = batch_steps(knobs, forms)
    n = min(args.steps, args.batch_steps)
    runs, sec = timed(steps, forms[0], n, min(args.warmup, 1))
    res = runs[-1][0]
    count = sum(r.count for r in res)
    comp = compare_forms(steps, forms[1:], result_key(res), n, min(args.warmup, 1), sec, count)
    return {"workload": spec["desc"], "form": forms[0], "value": count / sec, "unit": "cliques/s",
            "ms_per_step": round(sec * 1e3, 3), "steps": n, "count": count,
            "kernel_ms": round(runs[-1][1]["kernel_ns"] / 1e6, 3), "autotuned": rep, "compare": comp}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--form", default=None,
                    choices=["plain", "learned", "l2", "batched", "batched_learned", "sequential"])
    ap.add_argument("--compare", default=None,
                    help="comma-separated forms also timed in this run, at equal results ('' for none)")
    ap.add_argument("--compare-steps", type=int, default=10, help="at most this many timed steps per compared form")
    ap.add_argument("--batch", choices=["on", "off"], default="on",
                    help="with a single-graph workload, also time the 4096-graph batch section")
    ap.add_argument("--batch-steps", type=int, default=5, help="at most this many timed steps per batch form")
    ap.add_argument("--window", type=int, default=None, help="override the core window c")
    ap.add_argument("--no-worker-list", action="store_true")
    ap.add_argument("--bitmap-max-p", type=int, default=0)
    ap.add_argument("--wg-per-cu", type=int, default=0)
    ap.add_argument("--donate-min-p", type=int, default=0)
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--cpu-sample-mod", type=int, default=0, help="0: the workload's default sample")
    ap.add_argument("--peel-steps", action="store_true",
                    help="peel with graph-replayed step kernels instead of one cooperative launch "
                         "(for profilers that do not follow cooperative launches)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="launch one elementwise kernel that reads and writes 1 GiB each, as the "
                         "reference for scaling hardware byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print("this build runs on exactly one GPU: --gpus must be 1 (there is no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2212_01473_amd import mce

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    mce.load_library()
    spec = WORKLOADS[args.workload]
    form = args.form or spec["form"]
    compare = [f for f in (spec["compare"] if args.compare is None else args.compare).split(",") if f and f != form]
    c = spec["c"] if args.window is None else args.window
    knobs = dict(worker_list=not args.no_worker_list, bitmap_max_p=args.bitmap_max_p, wg_per_cu=args.wg_per_cu,
                 donate_min_p=args.donate_min_p, timeout_ms=600000)

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] calibration kernel: 1 GiB read + 1 GiB written")

    if spec["kind"] == "graph":
        g, steps = graph_steps(args.workload, c, knobs, [form] + compare,
                               load_kw=dict(peel_steps=True) if args.peel_steps else None)
        units = g.n
    else:
        g, steps, _ = batch_steps(knobs, [form] + compare)
        units = len(g)
    for f in [form] + compare:
        if f not in steps:
            raise SystemExit(f"form {f} does not apply to workload {args.workload}")

    runs, sec = timed(steps, form, args.steps, args.warmup)
    res, st, info = runs[-1]
    key = result_key(res)
    count = sum(r.count for r in res)
    for i, (rr, s, _) in enumerate(runs):
        log(f"[bench] {form} step {i}: count={sum(r.count for r in rr)} kernel={s['kernel_ns'] / 1e6:.2f}ms "
            f"setup={s['setup_ns'] / 1e6:.2f}ms nodes={s['nodes']} donations={s['donations']}")
    comp = compare_forms(steps, compare, key, min(args.steps, args.compare_steps), min(args.warmup, 1), sec, count)

    kern_ms = sum(s["kernel_ns"] for _, s, _ in runs) / len(runs) / 1e6
    cfg = {"workload": spec["desc"] if args.window is None else f"{args.workload} c={c}", "form": form,
           "count": count, "units": units}
    if info is not None:
        cfg.update({"n": int(info.n), "degeneracy": int(info.degeneracy), "max_degree": int(info.max_degree),
                    "core_window": c if c != FULL else "full", "hash": f"{res[0].hash:#018x}",
                    "max_clique": res[0].max_size, "peel_mode": int(info.peel_mode)})
    cfg.update({"workgroups": st["workgroups"], "tree_nodes": st["nodes"], "donations": st["donations"],
                "kernel_ms": round(kern_ms, 3), "setup_ms": round(st["setup_ns"] / 1e6, 3)})
    roof, others = rooflines(args.workload, c, st, kern_ms)
    out = {
        "metric": "maximal cliques/sec (wall time per step in ms_per_step); learned vs plain form",
        "value": count / sec,
        "unit": "cliques/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32/u64 (exact integer)",
        "data": "synthetic (seeded generator)",
        "config": cfg,
        "compare": comp,
        "roofline": roof,
        "roofline_other": others,
    }
    if spec["kind"] == "graph" and args.batch == "on":
        out["batch"] = batch_section(args, knobs)
    if args.cpu_baseline == "on":
        log("[bench] timing the CPU oracle on a sample")
        mod = args.cpu_sample_mod or spec["cpu_mod"]
        if spec["kind"] == "graph":
            out["cpu_baseline"] = cpu_baseline_graph(g, c, mod)
        else:
            out["cpu_baseline"] = cpu_baseline_batch(g, mod)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
