"""MI355X epsilon-graph library: Python binding of the C ABI in
``include/fnn.h`` (argument marshalling only; every step of the path runs in
the HIP kernels of ``libfnn.so``).

    import torch, paper_2510_14147_amd as fnn
    tree = fnn.fnn_tree_build(points_cuda, "l2")        # cover tree on the GPU
    g = fnn.fnn_eps_graph(tree, eps)                     # symmetric CSR
    g.row_ptr, g.col, g.dist                             # torch tensors (cuda)

PyTorch provides device memory (the caching allocator backs every array the
library hands back) and the stream (the current torch stream).  If the
compiled library is missing the import still works but every call raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfnn.so")

METRICS = {"l2": 0, "angular": 1, "hamming": 2, "levenshtein": 3}
PRECISIONS = {"fp32": 0, "bf16": 1, "fp8": 2, "i8": 3, "auto": 4, "fp16": 5}
SCHEDS = {"two_pass": 0, "learned": 1}

FNN_OK, FNN_EINVAL, FNN_ENOMEM, FNN_EHIP, FNN_EUNSUPPORTED, FNN_EINTERNAL = \
    0, -1, -2, -3, -4, -5


class FnnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fnn error {code}: {msg}")
        self.code = code


class fnn_options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("zeta", ctypes.c_int32),
                ("pack", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("kmax", ctypes.c_int32), ("trace", ctypes.c_int32),
                ("slack_pct", ctypes.c_int32), ("graph_passes", ctypes.c_int32),
                ("proj", ctypes.c_int32), ("list_cap", ctypes.c_int32),
                ("lpt", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


class fnn_tune_result(ctypes.Structure):
    _fields_ = [("best", fnn_options), ("best_ms", ctypes.c_double),
                ("base_ms", ctypes.c_double), ("ncand", ctypes.c_int32),
                ("cached", ctypes.c_int32), ("reserved", ctypes.c_double * 4)]


class fnn_csr(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("pad_", ctypes.c_uint32),
                ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("dist", ctypes.c_void_p)]


_STAT_I64 = ["n", "nodes", "leaf_blocks", "packs", "rounds", "netsel_passes",
             "build_dist_evals", "traverse_tests", "interactions",
             "tile_pairs", "filter_pairs", "filter_survivors",
             "fp64_rechecks", "edges", "overflow_rows", "validate_mismatch",
             "spilled"]
_STAT_F64 = ["max_rel_err", "build_ms", "traverse_ms", "tile_ms", "count_ms",
             "scan_ms", "fill_ms", "sort_ms", "total_ms", "pred_mae",
             "pred_sum_ratio", "filter_ms"]


class fnn_stats(ctypes.Structure):
    _fields_ = ([(k, ctypes.c_int64) for k in _STAT_I64] +
                [(k, ctypes.c_double) for k in _STAT_F64] +
                [("proj_dim", ctypes.c_int64), ("proj_captured", ctypes.c_double),
                 ("precision_used", ctypes.c_int64),
                 ("landmark_cells", ctypes.c_int64), ("landmark_rows", ctypes.c_int64),
                 ("landmark_partition_ms", ctypes.c_double),
                 ("landmark_forest_ms", ctypes.c_double),
                 ("landmark_merge_ms", ctypes.c_double),
                 ("launches", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                 ("graph_kernels", ctypes.c_int64),
                 ("fill_path", ctypes.c_int64)])


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None
_lock = threading.Lock()
_live = {}          # device pointer -> torch tensor owning it


def _torch():
    import torch
    return torch


@_ALLOC_FN
def _alloc_cb(nbytes, ctx):
    # an exception escaping a ctypes callback leaves its return value
    # undefined (not NULL): report every failure as NULL, which the library
    # turns into FNN_ENOMEM
    try:
        torch = _torch()
        t = torch.empty(int(nbytes), dtype=torch.uint8, device="cuda")
        p = t.data_ptr()
        _live[p] = t
        return p
    except BaseException:
        return None


@_FREE_FN
def _free_cb(ptr, ctx):
    _live.pop(ptr, None)


def lib():
    """Load libfnn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libfnn.so is not built; run python -c 'import __graft_entry__ as g; g.build()'")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.fnn_version.restype = ctypes.c_int
        L.fnn_last_error.restype = ctypes.c_char_p
        L.fnn_set_stream.argtypes = [vp]
        L.fnn_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
        L.fnn_tree_build_ex.argtypes = [vp, i64, i32, ctypes.c_int,
                                        ctypes.POINTER(fnn_options),
                                        ctypes.POINTER(vp)]
        L.fnn_tree_build.argtypes = [vp, i64, i32, ctypes.c_int,
                                     ctypes.POINTER(vp)]
        L.fnn_eps_graph_ex.argtypes = [vp, ctypes.c_double,
                                       ctypes.POINTER(fnn_options),
                                       ctypes.POINTER(ctypes.POINTER(fnn_csr))]
        L.fnn_eps_graph.argtypes = [vp, ctypes.c_double,
                                    ctypes.POINTER(ctypes.POINTER(fnn_csr))]
        L.fnn_eps_query.argtypes = [vp, vp, i64, ctypes.c_double,
                                    ctypes.POINTER(fnn_options),
                                    ctypes.POINTER(ctypes.POINTER(fnn_csr))]
        L.fnn_landmark_eps_graph.argtypes = [vp, i64, i32, ctypes.c_int, ctypes.c_double,
                                             i32, ctypes.c_uint64,
                                             ctypes.POINTER(fnn_options),
                                             ctypes.POINTER(ctypes.POINTER(fnn_csr))]
        L.fnn_tree_build_batch.argtypes = [vp, ctypes.POINTER(i64), i32, i32,
                                           ctypes.c_int, ctypes.POINTER(fnn_options),
                                           ctypes.POINTER(vp)]
        L.fnn_eps_graph_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i32,
                                          ctypes.POINTER(fnn_options),
                                          ctypes.POINTER(ctypes.POINTER(fnn_csr))]
        L.fnn_autotune.argtypes = [vp, ctypes.POINTER(i64), i32, i32, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(fnn_options), i32,
                                   ctypes.POINTER(fnn_tune_result)]
        L.fnn_autotune_clear.argtypes = []
        L.fnn_autotune_clear.restype = None
        L.fnn_free.argtypes = [vp]
        L.fnn_free.restype = None
        L.fnn_get_stats.argtypes = [vp, ctypes.POINTER(fnn_stats)]
        L.fnn_tree_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.fnn_tree_export.argtypes = [vp] + [vp] * 8
        L.fnn_set_cost_model.argtypes = [vp, i64]
        L.fnn_get_trace.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                    ctypes.POINTER(i64)]
        L.fnn_mlp_forward.argtypes = [vp, vp, i64, vp]
        L.fnn_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp,
                                        ctypes.POINTER(ctypes.c_double)]
        L.fnn_mlp_loss_grad_noalloc.argtypes = [vp, vp, vp, i64, vp, vp]
        L.fnn_mlp_train.argtypes = [vp, vp, vp, i64, i32, i32, ctypes.c_float,
                                    ctypes.c_uint64, vp]
        _lib = L
        L.fnn_set_allocator(_alloc_cb, _free_cb, None)
    return _lib


def _check(rc):
    if rc != FNN_OK:
        raise FnnError(rc, lib().fnn_last_error().decode())


def _bind_stream():
    torch = _torch()
    lib().fnn_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def _options(**kw) -> fnn_options:
    o = fnn_options()
    o.struct_size = ctypes.sizeof(fnn_options)
    for k, v in kw.items():
        if v is None:
            continue
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "sched" and isinstance(v, str):
            v = SCHEDS[v]
        setattr(o, k, int(v))
    return o


def _stats(handle) -> dict:
    s = fnn_stats()
    _check(lib().fnn_get_stats(handle, ctypes.byref(s)))
    return {k: getattr(s, k) for k in _STAT_I64 + _STAT_F64 +
            ["proj_dim", "proj_captured", "precision_used", "landmark_cells",
             "landmark_rows", "landmark_partition_ms", "landmark_forest_ms",
             "landmark_merge_ms", "launches", "graph_launches", "graph_kernels",
             "fill_path"]}


class Tree:
    """A device-resident cover tree (fnn_tree handle)."""

    def __init__(self, handle, n, dim, metric):
        self.handle, self.n, self.dim, self.metric = handle, n, dim, metric

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def free(self):
        if self.handle:
            lib().fnn_free(self.handle)
            self.handle = None

    @property
    def stats(self):
        return _stats(self.handle)


class Graph:
    """Symmetric CSR epsilon-graph; row_ptr int64 [n+1], col int32 [nnz],
    dist float32 [nnz] are torch tensors on the device."""

    def __init__(self, ptr):
        torch = _torch()
        self._ptr = ptr
        c = ptr.contents
        self.n, self.nnz = int(c.n), int(c.nnz)
        self.row_ptr = _live[c.row_ptr][: 8 * (self.n + 1)].view(torch.int64)
        self.col = _live[c.col][: 4 * self.nnz].view(torch.int32)
        self.dist = _live[c.dist][: 4 * self.nnz].view(torch.float32)
        self.stats = _stats(ptr)
        self.features = self.targets = None
        f, t, nn = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int64()
        if lib().fnn_get_trace(ctypes.cast(ptr, ctypes.c_void_p), ctypes.byref(f),
                               ctypes.byref(t), ctypes.byref(nn)) == FNN_OK:
            self.features = _live[f.value][: 4 * MLP_NFEAT * self.n].view(
                torch.float32).view(self.n, MLP_NFEAT)
            self.targets = _live[t.value][: 8 * self.n].view(torch.float32).view(
                self.n, 2)

    def free(self):
        if self._ptr:
            lib().fnn_free(ctypes.cast(self._ptr, ctypes.c_void_p))
            self._ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    def to_numpy(self):
        return (self.row_ptr.cpu().numpy(), self.col.cpu().numpy(),
                self.dist.cpu().numpy())


def _as_device_points(points, metric: str):
    torch = _torch()
    if metric in ("l2", "angular"):
        t = torch.as_tensor(points, dtype=torch.float32)
        if t.dim() != 2:
            raise ValueError("points must be [n, dim]")
        return t.to("cuda").contiguous(), t.shape[1]
    if metric == "hamming":
        if isinstance(points, np.ndarray):
            t = torch.from_numpy(np.ascontiguousarray(points).view(np.int64))
        else:
            t = points
        return t.to("cuda").contiguous(), t.shape[1] * 64
    if isinstance(points, np.ndarray):
        t = torch.from_numpy(np.ascontiguousarray(points, dtype=np.uint8))
    else:
        t = points
    return t.to("cuda").contiguous(), t.shape[1]


def fnn_tree_build(points, metric: str = "l2", zeta=None, pack=None,
                   kmax=None, graph_passes=None) -> Tree:
    """Cover tree of ``points`` (numpy array or tensor; moved to the GPU)."""
    m = METRICS[metric]
    t, dim = _as_device_points(points, metric)
    _bind_stream()
    h = ctypes.c_void_p()
    o = _options(zeta=zeta, pack=pack, kmax=kmax, graph_passes=graph_passes)
    _check(lib().fnn_tree_build_ex(ctypes.c_void_p(t.data_ptr()), t.shape[0],
                                   dim, m, ctypes.byref(o), ctypes.byref(h)))
    tree = Tree(h, t.shape[0], dim, metric)
    return tree


def fnn_tree_build_batch(points, offsets, metric: str = "l2", zeta=None,
                         pack=None, kmax=None, graph_passes=None) -> Tree:
    """One forest over many clouds: ``points`` holds the clouds' rows back to
    back, cloud c = rows [offsets[c], offsets[c+1])."""
    m = METRICS[metric]
    t, dim = _as_device_points(points, metric)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.size < 2:
        raise ValueError("offsets must hold nclouds + 1 values")
    if int(off[-1]) != t.shape[0]:
        raise ValueError("offsets[-1] must equal the number of rows")
    _bind_stream()
    h = ctypes.c_void_p()
    o = _options(zeta=zeta, pack=pack, kmax=kmax, graph_passes=graph_passes)
    _check(lib().fnn_tree_build_batch(
        ctypes.c_void_p(t.data_ptr()),
        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), off.size - 1, dim, m,
        ctypes.byref(o), ctypes.byref(h)))
    tree = Tree(h, t.shape[0], dim, metric)
    tree.nclouds = off.size - 1
    return tree


def fnn_eps_graph_batch(tree: Tree, eps, precision="fp32", sched="two_pass",
                        validate=False, trace=False, slack_pct=None,
                        proj=None, list_cap=None, lpt=False, graph_passes=None) -> Graph:
    """Per-cloud thresholds ``eps[c]``; one block-diagonal CSR over all rows."""
    if sched == "learned" and not _model_set and os.path.exists(COST_MODEL_PATH):
        fnn_set_cost_model(load_cost_model())
    e = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).ravel())
    _bind_stream()
    out = ctypes.POINTER(fnn_csr)()
    o = _options(precision=precision, sched=sched, validate=int(validate),
                 trace=int(trace), slack_pct=slack_pct, proj=proj, list_cap=list_cap,
                 lpt=int(lpt), graph_passes=graph_passes)
    _check(lib().fnn_eps_graph_batch(
        tree.handle, e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), e.size,
        ctypes.byref(o), ctypes.byref(out)))
    return Graph(out)


_OPT_KEYS = ("zeta", "pack", "precision", "sched", "kmax", "graph_passes", "proj", "lpt")


def fnn_autotune(points, offsets, metric: str, eps, reps: int = 2, **base) -> dict:
    """Fastest options for this input (see fnn_autotune in fnn.h).  A single
    cloud is offsets = [0, n].  Returns the options as keyword arguments of
    the build / query calls, with the timings."""
    # the learned schedule is a candidate when the shipped cost model exists
    if not _model_set and os.path.exists(COST_MODEL_PATH):
        fnn_set_cost_model(load_cost_model())
    m = METRICS[metric]
    t, dim = _as_device_points(points, metric)
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    e = np.ascontiguousarray(np.atleast_1d(np.asarray(eps, dtype=np.float64)))
    if off.size - 1 != e.size or int(off[-1]) != t.shape[0]:
        raise ValueError("offsets / eps do not match the points")
    _bind_stream()
    o = _options(**base)
    r = fnn_tune_result()
    _check(lib().fnn_autotune(
        ctypes.c_void_p(t.data_ptr()),
        off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), off.size - 1, dim, m,
        e.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(o),
        int(reps), ctypes.byref(r)))
    inv_p = {v: k for k, v in PRECISIONS.items()}
    inv_s = {v: k for k, v in SCHEDS.items()}
    best = {k: getattr(r.best, k) for k in _OPT_KEYS}
    best["precision"] = inv_p[best["precision"]]
    best["sched"] = inv_s[best["sched"]]
    return {"best": best, "best_ms": r.best_ms, "base_ms": r.base_ms,
            "ncand": r.ncand, "cached": bool(r.cached)}


def fnn_autotune_clear() -> None:
    lib().fnn_autotune_clear()


MLP_NPARAMS, MLP_NFEAT = 5378, 16
COST_MODEL_PATH = os.path.join(_HERE, "cost_model.json")
_model_set = False


def fnn_set_cost_model(params) -> None:
    """Install the cost model (5378 floats) used by sched="learned"."""
    global _model_set
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
    _check(lib().fnn_set_cost_model(ctypes.c_void_p(a.ctypes.data), a.size))
    _model_set = True


def load_cost_model(path: str = COST_MODEL_PATH) -> np.ndarray:
    import json
    with open(path) as f:
        return np.asarray(json.load(f)["params"], dtype=np.float32)


def fnn_eps_graph(tree: Tree, eps: float, precision="fp32",
                  sched="two_pass", validate=False, trace=False,
                  slack_pct=None, proj=None, list_cap=None, lpt=False,
                  graph_passes=None) -> Graph:
    """proj: filter on leading principal coordinates (None / 0 automatic,
    -1 off, else their number, a multiple of 16).  list_cap: initial
    survivor / edge list capacity (None: automatic; small values force the
    overflow paths).  graph_passes: traversal levels per replayed graph (1:
    every level eager)."""
    if sched == "learned" and not _model_set and os.path.exists(COST_MODEL_PATH):
        fnn_set_cost_model(load_cost_model())
    _bind_stream()
    out = ctypes.POINTER(fnn_csr)()
    o = _options(precision=precision, sched=sched, validate=int(validate),
                 trace=int(trace), slack_pct=slack_pct, proj=proj, list_cap=list_cap,
                 lpt=int(lpt), graph_passes=graph_passes)
    _check(lib().fnn_eps_graph_ex(tree.handle, float(eps), ctypes.byref(o),
                                  ctypes.byref(out)))
    return Graph(out)


def fnn_eps_query(tree: Tree, queries, eps: float, precision="fp32",
                  sched="two_pass", validate=False, proj=None, zeta=None,
                  pack=None, kmax=None, graph_passes=None) -> Graph:
    """Bichromatic range query: rows of ``queries`` (the tree's metric and
    dim) against the tree's points; a CSR with one row per query, columns =
    the tree's input indices."""
    t, dim = _as_device_points(queries, tree.metric)
    if dim != tree.dim:
        raise ValueError(f"queries have dim {dim}, the tree {tree.dim}")
    _bind_stream()
    out = ctypes.POINTER(fnn_csr)()
    o = _options(precision=precision, sched=sched, validate=int(validate), proj=proj,
                 zeta=zeta, pack=pack, kmax=kmax, graph_passes=graph_passes)
    _check(lib().fnn_eps_query(tree.handle, ctypes.c_void_p(t.data_ptr()), t.shape[0],
                               float(eps), ctypes.byref(o), ctypes.byref(out)))
    return Graph(out)


def fnn_landmark_eps_graph(points, eps: float, ncells: int, metric: str = "l2",
                           seed: int = 0, precision="fp32", sched="two_pass",
                           zeta=None, pack=None, kmax=None, proj=None) -> Graph:
    """The epsilon-graph by the landmark scheme: ``ncells`` seeded centres,
    Voronoi cells, eps-ghosts (Lemma 1), one batched forest over cells +
    ghosts, every ordered pair kept once.  Same CSR as fnn_eps_graph."""
    if sched == "learned" and not _model_set and os.path.exists(COST_MODEL_PATH):
        fnn_set_cost_model(load_cost_model())
    m = METRICS[metric]
    t, dim = _as_device_points(points, metric)
    _bind_stream()
    out = ctypes.POINTER(fnn_csr)()
    o = _options(precision=precision, sched=sched, zeta=zeta, pack=pack, kmax=kmax,
                 proj=proj)
    _check(lib().fnn_landmark_eps_graph(ctypes.c_void_p(t.data_ptr()), t.shape[0], dim, m,
                                        float(eps), int(ncells), ctypes.c_uint64(seed),
                                        ctypes.byref(o), ctypes.byref(out)))
    return Graph(out)


def fnn_free(obj):
    obj.free()


def fnn_get_stats(obj) -> dict:
    return obj.stats


def fnn_tree_export(tree: Tree) -> dict:
    """Host copy of the cover tree (layout of fnn_tree_export in fnn.h)."""
    n, nn = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().fnn_tree_info(tree.handle, ctypes.byref(n), ctypes.byref(nn)))
    n, nn = n.value, nn.value
    a = dict(order=np.zeros(n, np.int32), center=np.zeros(nn, np.int32),
             radius=np.zeros(nn, np.float32), level=np.zeros(nn, np.int32),
             child_begin=np.zeros(nn, np.int32), child_count=np.zeros(nn, np.int32),
             pt_begin=np.zeros(nn, np.int32), pt_end=np.zeros(nn, np.int32))
    _bind_stream()
    _check(lib().fnn_tree_export(tree.handle, *[ctypes.c_void_p(a[k].ctypes.data) for k in
                                                ("order", "center", "radius", "level",
                                                 "child_begin", "child_count",
                                                 "pt_begin", "pt_end")]))
    a["nnodes"] = nn
    return a


def version() -> int:
    return lib().fnn_version()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def fnn_mlp_forward(params, X):
    """Y[n,2] = f(X[n,16]) with the library's inference kernel (cuda
    float32 tensors)."""
    torch = _torch()
    Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device=X.device)
    _bind_stream()
    _check(lib().fnn_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(Y)))
    return Y


def fnn_mlp_loss_grad(params, X, T):
    """(loss, grad) of the full batch, from the library's backward kernel."""
    torch = _torch()
    g = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
    loss = ctypes.c_double()
    _bind_stream()
    _check(lib().fnn_mlp_loss_grad(_ptr(params), _ptr(X), _ptr(T), X.shape[0],
                                   _ptr(g), ctypes.byref(loss)))
    return loss.value, g


def fnn_mlp_loss_grad_noalloc(params, X, T, grad=None, loss=None):
    """The allocation-free gradient entry point: grad (5378 floats) and loss
    (one float64) are caller-provided cuda tensors (allocated here when not
    given); returns (loss tensor, grad tensor) without waiting on the
    stream."""
    torch = _torch()
    if grad is None:
        grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
    _bind_stream()
    _check(lib().fnn_mlp_loss_grad_noalloc(_ptr(params), _ptr(X), _ptr(T), X.shape[0],
                                           _ptr(grad), _ptr(loss)))
    return loss, grad


def fnn_mlp_train(params, X, T, epochs=4, batch=4096, lr=1e-3, seed=0):
    """Train params in place (Adam); returns the mean loss of each epoch."""
    losses = np.zeros(max(epochs, 1), dtype=np.float64)
    _bind_stream()
    _check(lib().fnn_mlp_train(_ptr(params), _ptr(X), _ptr(T), X.shape[0],
                               int(epochs), int(batch), ctypes.c_float(lr),
                               ctypes.c_uint64(seed),
                               ctypes.c_void_p(losses.ctypes.data)))
    return losses[:epochs]

