"""Training pipeline of the learned root ordering (orchestration only).

The cost model predicts log(1 + search-tree nodes) of a first-level subtree
from four cheap features.  Labels come from the plain enumeration itself: it
counts tree nodes per root (per-root statistics).  Features come from the
library's feature kernel; training runs the library's FP32 forward/backward
and Adam kernels; inference (in the enumeration) is BF16.  This module only
moves tensors between those calls and stores the weights.
"""
from __future__ import annotations

import math
import os

import numpy as np

from . import inputs as I
from . import mce

MODEL_FLOATS = mce.MODEL_FLOATS
IN, H = 4, 64


def init_model(seed: int = 0) -> np.ndarray:
    """Seeded uniform initialisation, scaled by fan-in (He et al. 2015 bounds
    for ReLU layers); mean 0 / std 1 normalisation until fitted."""
    rng = np.random.Generator(np.random.PCG64(seed))
    th = np.zeros(MODEL_FLOATS, dtype=np.float32)
    o = 0

    def fill(rows, cols, o):
        bound = math.sqrt(6.0 / cols)
        th[o:o + rows * cols] = rng.uniform(-bound, bound, rows * cols)
        return o + rows * cols

    o = fill(H, IN, o)
    o += H  # b1
    o = fill(H, H, o)
    o += H
    o = fill(H, H, o)
    o += H
    o = fill(1, H, o)
    o += 1  # b4
    th[o:o + IN] = 0.0
    th[o + IN:o + 2 * IN] = 1.0
    return th


def collect(g, c: int, timeout_ms: int = 300000):
    """(features, labels) on the device for the roots of graph g in window c
    that have a non-empty P: labels = log1p(tree nodes) measured by the plain
    enumeration."""
    import torch

    dev = "cuda"
    cnt = torch.zeros(g.n, dtype=torch.int64, device=dev)
    hsh = torch.zeros(g.n, dtype=torch.int64, device=dev)
    nodes = torch.zeros(g.n, dtype=torch.int64, device=dev)
    with mce.load_graph(g) as dg:
        mce.enumerate_cliques(dg, max_root_core=c, root_stats=(cnt, hsh, nodes), timeout_ms=timeout_ms)
        core, _, order = dg.order_arrays()
        rank = np.empty(g.n, dtype=np.int64)
        rank[order] = np.arange(g.n)
        deg = g.degrees()
        src = np.repeat(np.arange(g.n), deg)
        later = rank[g.col_idx.astype(np.int64)] > rank[src]
        outdeg = np.bincount(src[later], minlength=g.n)
        roots = np.flatnonzero((outdeg > 0) & (core <= c)).astype(np.int32)
        ids = torch.from_numpy(roots).to(dev)
        feat = mce.root_features(dg, ids).clone()
    label = torch.log1p(nodes[ids.long()].to(torch.float32))
    return feat, label


def train(feat, label, epochs: int = 400, lr: float = 3e-3, seed: int = 0):
    import torch

    model = torch.from_numpy(init_model(seed)).cuda()
    hist = mce.model_train(model, feat.contiguous(), label.contiguous(), epochs=epochs, lr=lr)
    return model, hist


TRAIN_GRAPHS = [
    # (scale, edge factor, seed, window as a fraction of the degeneracy):
    # R-MAT graphs with the workloads' quadrant probabilities and seeds other
    # than those of the measured workloads; the windows stop below each graph's
    # densest shell, where one plain run takes a few seconds at most
    (18, 16, 6, 0.7),
    (18, 32, 7, 0.7),
    (18, 16, 8, 0.7),
]


def default_training_set(graphs=TRAIN_GRAPHS):
    import torch

    feats, labels = [], []
    for scale, ef, seed, frac in graphs:
        g = I.rmat(scale, ef, 0.57, 0.19, 0.19, 0.05, seed)
        with mce.load_graph(g) as dg:
            c = int(frac * dg.info().degeneracy)
        f, l = collect(g, c)
        feats.append(f)
        labels.append(l)
    return torch.cat(feats), torch.cat(labels)


def save(model, path: str):
    arr = model.detach().cpu().numpy() if hasattr(model, "detach") else np.asarray(model)
    np.save(path, arr.astype(np.float32))


def load(path: str):
    import torch

    arr = np.load(path, allow_pickle=False).astype(np.float32)
    if arr.shape != (MODEL_FLOATS,):
        raise ValueError(f"model file {path} has shape {arr.shape}")
    return torch.from_numpy(arr).cuda()


def cached_model(path: str | None = None, epochs: int = 400):
    """Load the trained model, training (and storing) it first when absent."""
    path = path or os.path.join(I.cache_dir(), "mce_cost_model_r18.npy")
    if os.path.exists(path):
        return load(path)
    feat, label = default_training_set()
    model, _ = train(feat, label, epochs=epochs)
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        save(model, path)
    except OSError:
        pass
    return model
