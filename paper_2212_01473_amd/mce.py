"""Thin ctypes binding of the C ABI in ``include/mce.h``.

Argument marshalling only: every step of the enumeration runs in the HIP
library.  PyTorch is used for device memory and streams when given device
tensors.  Importing this module never falls back to anything else: when the
library is missing, ``load_library`` raises.
"""
from __future__ import annotations

import ctypes as C
from collections.abc import Sequence
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmce.so")
_lib = None

MCE_OK = 0
MCE_WARN_STREAM_TRUNCATED = 1
MCE_ERR_INVALID_ARG = -1
MCE_ERR_INVALID_GRAPH = -2
MCE_ERR_OUT_OF_MEMORY = -3
MCE_ERR_DEVICE = -4
MCE_ERR_BUFFER_TOO_SMALL = -5
MCE_ERR_TIMEOUT = -6
MCE_ERR_UNSUPPORTED = -7

MCE_LOAD_DEVICE_PTRS = 0x1
MCE_LOAD_NO_VALIDATE = 0x2
MCE_LOAD_PEEL_STEPS = 0x4

F_WORKER_LIST = 0x01
F_LEARNED_ORDER = 0x02
F_SPLIT = 0x04
GRAPH_WHOLE = 0xFFFFFFFF
F_STATS = 0x08
F_STREAM = 0x10
F_ROOT_STATS = 0x20
F_REVERSE_ORDER = 0x40
F_CUSTOM_ORDER = 0x80
F_TASK_LOG = 0x100
F_L2_ROOTS = 0x200

STAT_NAMES = ["nodes", "donations", "tasks", "roots", "workgroups", "kernel_ns", "setup_ns", "xtests",
              "build_edges", "hbm_row_tasks", "idle_ns", "lds_bytes", "probes", "root_words",
              "busy_ns", "max_task_ns", "xrow_tasks", "build_ns", "task_log", "donate_ns",
              "pop_fails", "xcol_words", "fold_donations"]

FULL = 0xFFFFFFFF

EXPORTED = ["mce_load_csr", "mce_load_csr_batch", "mce_graph_get_info", "mce_graph_copy_order", "mce_enumerate",
            "mce_enumerate_batch", "mce_free", "mce_status_string", "mce_last_error", "mce_version",
            "mce_root_features", "mce_model_predict", "mce_model_train", "mce_model_loss_grad",
            "mce_model_loss_grad_noalloc", "mce_autotune"]

MODEL_FLOATS = 8713
MCE_NOALLOC_MAX_SAMPLES = 16384  # include/mce.h


class MCEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class GraphInfo(C.Structure):
    _fields_ = [("n", C.c_uint32), ("nnz", C.c_uint64), ("max_degree", C.c_uint32),
                ("degeneracy", C.c_uint32), ("n_isolated", C.c_uint64), ("peel_rounds", C.c_uint32),
                ("max_out_degree", C.c_uint32), ("max_in_degree", C.c_uint32), ("n_graphs", C.c_uint32),
                ("peel_mode", C.c_uint32)]


class Options(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("flags", C.c_uint32), ("max_root_core", C.c_uint32),
                ("wg_per_cu", C.c_uint32), ("bitmap_max_p", C.c_uint32), ("donate_min_p", C.c_uint32),
                ("donate_max_depth", C.c_uint32), ("split_top", C.c_uint32), ("model", C.c_void_p),
                ("stream", C.c_void_p), ("timeout_ms", C.c_uint64), ("root_order", C.c_void_p),
                ("root_count", C.c_void_p), ("root_hash", C.c_void_p), ("root_nodes", C.c_void_p),
                ("xrow_ratio", C.c_uint32), ("xrow_min_u", C.c_uint32), ("xrow_budget_words", C.c_uint64),
                ("donate_every", C.c_uint32), ("task_log_min_us", C.c_uint32),
                ("task_log", C.c_void_p), ("task_log_cap", C.c_uint64)]


class TrainOptions(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("epochs", C.c_uint32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float), ("fit_norm", C.c_uint32), ("reserved", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("count", C.c_uint64), ("hash", C.c_uint64), ("max_clique_size", C.c_uint32),
                ("hist_len", C.c_uint32), ("hist", C.POINTER(C.c_uint64)),
                ("stream_vertices", C.c_void_p), ("stream_vcap", C.c_uint64),
                ("stream_offsets", C.c_void_p), ("stream_ocap", C.c_uint64),
                ("stream_vertices_written", C.c_uint64), ("stream_cliques_written", C.c_uint64),
                ("stats", C.c_uint64 * 24)]


class TuneReport(C.Structure):
    _fields_ = [("struct_size", C.c_uint32), ("passes", C.c_uint32), ("repeats", C.c_uint32),
                ("trials", C.c_uint32), ("base_ms", C.c_double), ("best_ms", C.c_double)]


def load_library(path: str | None = None):
    """Load libmce.so (built in-tree by ``build.py``); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run paper_2212_01473_amd/build.py)")
    lib = C.CDLL(path)
    u32p = C.c_void_p
    lib.mce_load_csr.restype = C.c_int
    lib.mce_load_csr.argtypes = [u32p, u32p, C.c_uint32, C.c_uint64, C.c_uint32, C.c_void_p,
                                 C.POINTER(C.c_void_p)]
    lib.mce_load_csr_batch.restype = C.c_int
    lib.mce_load_csr_batch.argtypes = [u32p, u32p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_uint32,
                                       C.c_void_p, C.POINTER(C.c_void_p)]
    lib.mce_graph_get_info.restype = C.c_int
    lib.mce_graph_get_info.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(GraphInfo)]
    lib.mce_graph_copy_order.restype = C.c_int
    lib.mce_graph_copy_order.argtypes = [C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.mce_enumerate.restype = C.c_int
    lib.mce_enumerate.argtypes = [C.c_void_p, C.POINTER(Options), C.POINTER(Result)]
    lib.mce_enumerate_batch.restype = C.c_int
    lib.mce_enumerate_batch.argtypes = [C.c_void_p, C.POINTER(Options), C.POINTER(Result), C.c_uint32]
    lib.mce_free.restype = None
    lib.mce_free.argtypes = [C.c_void_p]
    lib.mce_status_string.restype = C.c_char_p
    lib.mce_status_string.argtypes = [C.c_int]
    lib.mce_last_error.restype = C.c_char_p
    lib.mce_last_error.argtypes = []
    lib.mce_version.restype = C.c_char_p
    lib.mce_version.argtypes = []
    lib.mce_root_features.restype = C.c_int
    lib.mce_root_features.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.mce_model_predict.restype = C.c_int
    lib.mce_model_predict.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p]
    lib.mce_model_train.restype = C.c_int
    lib.mce_model_train.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.POINTER(TrainOptions),
                                    C.c_void_p, C.c_void_p]
    lib.mce_model_loss_grad.restype = C.c_int
    lib.mce_model_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                        C.POINTER(C.c_float), C.c_void_p]
    lib.mce_model_loss_grad_noalloc.restype = C.c_int
    lib.mce_model_loss_grad_noalloc.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                                C.POINTER(C.c_float), C.c_void_p]
    lib.mce_autotune.restype = C.c_int
    lib.mce_autotune.argtypes = [C.c_void_p, C.POINTER(Options), C.POINTER(Options), C.POINTER(TuneReport)]
    _lib = lib
    return lib


def _check(st: int, what: str):
    if st < 0:
        lib = load_library()
        raise MCEError(st, f"{what}: {lib.mce_status_string(st).decode()}: {lib.mce_last_error().decode()}")
    return st


def _torch_stream():
    try:
        import torch

        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:  # pragma: no cover - torch is plumbing only
        pass
    return C.c_void_p(None)


def _is_device_tensor(x) -> bool:
    return hasattr(x, "is_cuda") and bool(x.is_cuda)


@dataclass
class EnumResult:
    count: int
    hash: int
    hist: np.ndarray
    max_size: int
    stats: dict = field(default_factory=dict)
    status: int = 0
    stream_cliques: int = 0
    stream_vertices: int = 0


class Graph:
    """Library-owned device graph (mce_graph handle)."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self, idx: int = 0) -> GraphInfo:
        gi = GraphInfo()
        _check(load_library().mce_graph_get_info(self._h, idx, C.byref(gi)), "mce_graph_get_info")
        return gi

    def order_arrays(self, idx: int = 0):
        """(core, peel_round, order) as numpy arrays (input-id space)."""
        n = self.info(idx).n
        core = np.zeros(max(n, 1), dtype=np.uint32)
        rnd = np.zeros(max(n, 1), dtype=np.uint32)
        order = np.zeros(max(n, 1), dtype=np.uint32)
        _check(load_library().mce_graph_copy_order(self._h, idx, C.c_void_p(core.ctypes.data),
                                                   C.c_void_p(rnd.ctypes.data), C.c_void_p(order.ctypes.data)),
               "mce_graph_copy_order")
        return core[:n], rnd[:n], order[:n]

    def free(self):
        if self._h:
            load_library().mce_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.free()


def load_csr(row_ptr, col_idx, n: int | None = None, validate: bool = True, stream=None,
             peel_steps: bool = False) -> Graph:
    """Load a CSR graph from numpy arrays (host) or torch device tensors."""
    lib = load_library()
    flags = (0 if validate else MCE_LOAD_NO_VALIDATE) | (MCE_LOAD_PEEL_STEPS if peel_steps else 0)
    if _is_device_tensor(row_ptr):
        flags |= MCE_LOAD_DEVICE_PTRS
        nn = int(row_ptr.numel()) - 1 if n is None else n
        nnz = int(col_idx.numel())
        rp_p = C.c_void_p(row_ptr.data_ptr())
        ci_p = C.c_void_p(col_idx.data_ptr())
        keep = (row_ptr, col_idx)
    else:
        rp = np.ascontiguousarray(row_ptr, dtype=np.uint32)
        ci = np.ascontiguousarray(col_idx, dtype=np.uint32)
        nn = rp.shape[0] - 1 if n is None else n
        nnz = ci.shape[0]
        if ci.size == 0:
            ci = np.zeros(1, dtype=np.uint32)
        rp_p = C.c_void_p(rp.ctypes.data)
        ci_p = C.c_void_p(ci.ctypes.data)
        keep = (rp, ci)
    h = C.c_void_p()
    st = lib.mce_load_csr(rp_p, ci_p, nn, nnz, flags, stream if stream is not None else _torch_stream(),
                          C.byref(h))
    del keep
    _check(st, "mce_load_csr")
    return Graph(h)


def load_graph(g, validate: bool = True, peel_steps: bool = False) -> Graph:
    """Load an ``inputs.CSRGraph``."""
    return load_csr(g.row_ptr, g.col_idx, g.n, validate=validate, peel_steps=peel_steps)


def load_batch(graphs, validate: bool = True, peel_steps: bool = False) -> Graph:
    """mce_load_csr_batch from host arrays (a list of CSRGraph)."""
    from .inputs import concat_batch

    lib = load_library()
    rp, ci, row_off, col_off = concat_batch(graphs)
    if ci.size == 0:
        ci = np.zeros(1, dtype=np.uint32)
    h = C.c_void_p()
    flags = (0 if validate else MCE_LOAD_NO_VALIDATE) | (MCE_LOAD_PEEL_STEPS if peel_steps else 0)
    st = lib.mce_load_csr_batch(C.c_void_p(rp.ctypes.data), C.c_void_p(ci.ctypes.data),
                                C.c_void_p(row_off.ctypes.data), C.c_void_p(col_off.ctypes.data),
                                len(graphs), flags, _torch_stream(), C.byref(h))
    _check(st, "mce_load_csr_batch")
    return Graph(h)


def load_batch_device(rp_cat, ci_cat, row_off, col_off, validate: bool = True) -> Graph:
    """mce_load_csr_batch with MCE_LOAD_DEVICE_PTRS: rp_cat / ci_cat are device
    int32 tensors (concatenated CSRs), row_off / col_off host uint64 arrays."""
    lib = load_library()
    row_off = np.ascontiguousarray(row_off, dtype=np.uint64)
    col_off = np.ascontiguousarray(col_off, dtype=np.uint64)
    if not (_is_device_tensor(rp_cat) and _is_device_tensor(ci_cat)):
        raise TypeError("rp_cat and ci_cat must be device tensors")
    h = C.c_void_p()
    flags = MCE_LOAD_DEVICE_PTRS | (0 if validate else MCE_LOAD_NO_VALIDATE)
    st = lib.mce_load_csr_batch(C.c_void_p(rp_cat.data_ptr()), C.c_void_p(ci_cat.data_ptr()),
                                C.c_void_p(row_off.ctypes.data), C.c_void_p(col_off.ctypes.data),
                                len(row_off) - 1, flags, _torch_stream(), C.byref(h))
    _check(st, "mce_load_csr_batch")
    return Graph(h)


def make_options(max_root_core: int = FULL, worker_list: bool = True, flags: int = 0, wg_per_cu: int = 0,
                 model=None, split: bool = False, split_top: int = 0,
                 bitmap_max_p: int = 0, donate_min_p: int = 0, donate_max_depth: int = 0,
                 timeout_ms: int = 0, stream=None, root_order=None, root_stats=None, xrow_ratio: int = 0,
                 xrow_budget_words: int = 0, xrow_min_u: int = 0, donate_every: int = 0,
                 task_log=None, task_log_min_us: int = 0, l2_roots: bool = False) -> Options:
    o = Options()
    o.donate_every = donate_every
    o.xrow_ratio = xrow_ratio
    o.xrow_min_u = xrow_min_u
    o.xrow_budget_words = xrow_budget_words
    o.struct_size = C.sizeof(Options)
    o.flags = flags | (F_WORKER_LIST if worker_list else 0) | F_STATS | (F_L2_ROOTS if l2_roots else 0)
    if model is not None:
        o.flags |= F_LEARNED_ORDER | (F_SPLIT if split else 0)
        o.model = C.c_void_p(model.data_ptr())
        o.split_top = split_top
    elif split:
        raise ValueError("split needs a model")
    o.max_root_core = int(max_root_core) & 0xFFFFFFFF
    o.wg_per_cu = wg_per_cu
    o.bitmap_max_p = bitmap_max_p
    o.donate_min_p = donate_min_p
    o.donate_max_depth = donate_max_depth
    o.timeout_ms = timeout_ms
    o.stream = stream if stream is not None else _torch_stream()
    if root_order is not None:
        o.flags |= F_CUSTOM_ORDER
        o.root_order = C.c_void_p(root_order.data_ptr())
    if task_log is not None:
        # device int64 tensor [cap, 8]
        o.flags |= F_TASK_LOG
        o.task_log = C.c_void_p(task_log.data_ptr())
        o.task_log_cap = int(task_log.shape[0])
        o.task_log_min_us = task_log_min_us
    if root_stats is not None:
        cnt, hsh, nodes = root_stats
        o.flags |= F_ROOT_STATS
        o.root_count = C.c_void_p(cnt.data_ptr())
        o.root_hash = C.c_void_p(hsh.data_ptr())
        o.root_nodes = C.c_void_p(nodes.data_ptr())
    return o


def _to_result(r: Result, hist: np.ndarray, st: int) -> EnumResult:
    top = int(r.max_clique_size)
    stats = {name: int(r.stats[i]) for i, name in enumerate(STAT_NAMES)}
    return EnumResult(count=int(r.count), hash=int(r.hash), hist=hist[: top + 1].copy() if hist.size else hist,
                      max_size=top, stats=stats, status=st, stream_cliques=int(r.stream_cliques_written),
                      stream_vertices=int(r.stream_vertices_written))


def enumerate_cliques(g: Graph, hist_len: int | None = None, options: Options | None = None,
                      stream_buffers=None, **kw) -> EnumResult:
    """Run mce_enumerate; kwargs build an Options when none is given."""
    lib = load_library()
    opt = options if options is not None else make_options(**kw)
    if hist_len is None:
        hist_len = g.info().degeneracy + 2
    hist = np.zeros(max(hist_len, 1), dtype=np.uint64)
    r = Result()
    r.hist_len = hist_len
    r.hist = hist.ctypes.data_as(C.POINTER(C.c_uint64))
    if stream_buffers is not None:
        verts, offs = stream_buffers
        opt.flags |= F_STREAM
        r.stream_vertices = C.c_void_p(verts.data_ptr())
        r.stream_vcap = int(verts.numel())
        r.stream_offsets = C.c_void_p(offs.data_ptr())
        r.stream_ocap = int(offs.numel())
    st = lib.mce_enumerate(g.handle, C.byref(opt), C.byref(r))
    _check(st, "mce_enumerate")
    return _to_result(r, hist, st)


# numpy view of an array of mce_result (same layout as Result), so a batch's
# results are marshalled without a Python loop over the graphs
_RESULT_DTYPE = np.dtype({
    "names": ["count", "hash", "max_clique_size", "hist_len", "hist", "stats"],
    "formats": [np.uint64, np.uint64, np.uint32, np.uint32, np.uint64, (np.uint64, 24)],
    "offsets": [Result.count.offset, Result.hash.offset, Result.max_clique_size.offset, Result.hist_len.offset,
                Result.hist.offset, Result.stats.offset],
    "itemsize": C.sizeof(Result)})


class BatchResults(Sequence):
    """The per-graph results of mce_enumerate_batch: graph i's EnumResult is
    built when indexed; counts, hashes and the histogram matrix are arrays."""

    def __init__(self, rec: np.ndarray, hist: np.ndarray, status: int):
        self._rec, self._hist, self._status = rec, hist, status

    def __len__(self) -> int:
        return len(self._rec)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self[j] for j in range(*i.indices(len(self)))]
        r = self._rec[i]
        top = int(r["max_clique_size"])
        stats = {name: int(r["stats"][k]) for k, name in enumerate(STAT_NAMES)}
        return EnumResult(count=int(r["count"]), hash=int(r["hash"]), hist=self._hist[i, : top + 1].copy(),
                          max_size=top, stats=stats, status=self._status)

    @property
    def counts(self) -> np.ndarray:
        return self._rec["count"].copy()

    @property
    def hashes(self) -> np.ndarray:
        return self._rec["hash"].copy()


def enumerate_batch(g: Graph, options: Options | None = None, **kw) -> BatchResults:
    lib = load_library()
    info = g.info(GRAPH_WHOLE)
    ng = info.n_graphs
    opt = options if options is not None else make_options(**kw)
    hl = info.degeneracy + 2  # the largest member degeneracy + 2 serves every member
    hist = np.zeros((ng, hl), dtype=np.uint64)
    rec = np.zeros(ng, dtype=_RESULT_DTYPE)
    rec["hist_len"] = hl
    rec["hist"] = hist.ctypes.data + np.arange(ng, dtype=np.uint64) * np.uint64(hl * 8)
    st = lib.mce_enumerate_batch(g.handle, C.byref(opt), C.cast(rec.ctypes.data, C.POINTER(Result)), ng)
    _check(st, "mce_enumerate_batch")
    return BatchResults(rec, hist, st)


def autotune(g: Graph, passes: int = 1, repeats: int = 1, options: Options | None = None, **kw):
    """mce_autotune on a single-graph or batch handle: (tuned Options, report dict)."""
    lib = load_library()
    base = options if options is not None else make_options(**kw)
    tuned = Options()
    rep = TuneReport()
    rep.struct_size = C.sizeof(TuneReport)
    rep.passes = passes
    rep.repeats = repeats
    _check(lib.mce_autotune(g.handle, C.byref(base), C.byref(tuned), C.byref(rep)), "mce_autotune")
    knobs = {k: int(getattr(tuned, k)) for k in ("donate_min_p", "bitmap_max_p", "wg_per_cu", "donate_max_depth",
                                                  "xrow_ratio")}
    return tuned, dict(trials=int(rep.trials), base_ms=float(rep.base_ms), best_ms=float(rep.best_ms), **knobs)


def version() -> str:
    return load_library().mce_version().decode()


# ---------------------------------------------------------------- learned cost model

def root_features(g: Graph, root_ids):
    """Device float32 [n, 4] features of the given roots (device int32 input ids)."""
    import torch

    n = int(root_ids.numel())
    feat = torch.empty((max(n, 1), 4), dtype=torch.float32, device=root_ids.device)
    _check(load_library().mce_root_features(g.handle, C.c_void_p(root_ids.data_ptr()), n,
                                            C.c_void_p(feat.data_ptr()), _torch_stream()), "mce_root_features")
    return feat[:n]


def model_predict(model, feat):
    import torch

    n = int(feat.shape[0])
    out = torch.empty(max(n, 1), dtype=torch.float32, device=feat.device)
    _check(load_library().mce_model_predict(C.c_void_p(model.data_ptr()), C.c_void_p(feat.data_ptr()), n,
                                            C.c_void_p(out.data_ptr()), _torch_stream()), "mce_model_predict")
    return out[:n]


def model_loss_grad(model, feat, target):
    import torch

    grad = torch.empty(MODEL_FLOATS, dtype=torch.float32, device=feat.device)
    loss = C.c_float()
    _check(load_library().mce_model_loss_grad(C.c_void_p(model.data_ptr()), C.c_void_p(feat.data_ptr()),
                                              C.c_void_p(target.data_ptr()), int(feat.shape[0]),
                                              C.c_void_p(grad.data_ptr()), C.byref(loss), _torch_stream()),
           "mce_model_loss_grad")
    return grad, float(loss.value)


def model_loss_grad_noalloc(model, feat, target, grad) -> float:
    """mce_model_loss_grad_noalloc: the gradient into the caller's device
    tensor grad (float32[MODEL_FLOATS]); returns the loss."""
    loss = C.c_float()
    _check(load_library().mce_model_loss_grad_noalloc(C.c_void_p(model.data_ptr()), C.c_void_p(feat.data_ptr()),
                                                      C.c_void_p(target.data_ptr()), int(feat.shape[0]),
                                                      C.c_void_p(grad.data_ptr()), C.byref(loss), _torch_stream()),
           "mce_model_loss_grad_noalloc")
    return float(loss.value)


def model_train(model, feat, target, epochs: int = 300, lr: float = 3e-3, beta1: float = 0.9,
                beta2: float = 0.999, eps: float = 1e-8, fit_norm: bool = True) -> np.ndarray:
    """Train in place (FP32 kernels, full-batch Adam); returns the loss per epoch."""
    o = TrainOptions()
    o.struct_size = C.sizeof(TrainOptions)
    o.epochs = epochs
    o.lr, o.beta1, o.beta2, o.eps = lr, beta1, beta2, eps
    o.fit_norm = 1 if fit_norm else 0
    hist = np.zeros(epochs, dtype=np.float32)
    _check(load_library().mce_model_train(C.c_void_p(model.data_ptr()), C.c_void_p(feat.data_ptr()),
                                          C.c_void_p(target.data_ptr()), int(feat.shape[0]), C.byref(o),
                                          C.c_void_p(hist.ctypes.data), _torch_stream()), "mce_model_train")
    return hist
