"""Python access to the CPU oracle (``liboracle.so``, built from
``fnn_oracle.c`` by ``oracle/build.py``).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg use it; the GPU library never does.

Metric ids: 0 = L2, 1 = angular, 2 = Hamming, 3 = Levenshtein.
Point layouts are those of ``paper_2510_14147_amd.datagen``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

L2, ANGULAR, HAMMING, LEVENSHTEIN = 0, 1, 2, 3

_i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
_vp = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b  # noqa: F401  (package-relative build)
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.orc_l2_sq.restype = ctypes.c_double
        L.orc_l2_sq.argtypes = [_f32p, _f32p, ctypes.c_int32]
        L.orc_ang_terms.restype = None
        L.orc_ang_terms.argtypes = [_f32p, _f32p, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
        L.orc_ang_pred.restype = ctypes.c_int
        L.orc_ang_pred.argtypes = [ctypes.c_double] * 4
        L.orc_ang_dist.restype = ctypes.c_double
        L.orc_ang_dist.argtypes = [_f32p, _f32p, ctypes.c_int32]
        L.orc_ham.restype = ctypes.c_int32
        L.orc_ham.argtypes = [_u64p, _u64p, ctypes.c_int32]
        L.orc_lev.restype = ctypes.c_int32
        L.orc_lev.argtypes = [_u8p, ctypes.c_int32, _u8p, ctypes.c_int32]
        L.orc_lev_banded.restype = ctypes.c_int32
        L.orc_lev_banded.argtypes = [_u8p, ctypes.c_int32, _u8p,
                                     ctypes.c_int32, ctypes.c_int32]
        L.orc_eps_param.restype = ctypes.c_double
        L.orc_eps_param.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_bf_count.restype = ctypes.c_int64
        L.orc_bf_count.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_double, _vp,
                                   ctypes.c_int64, _i64p]
        L.orc_bf_fill.restype = None
        L.orc_bf_fill.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_double, _vp,
                                  ctypes.c_int64, _i64p, _i32p, _f64p]
        L.orc_rows_dist.restype = None
        L.orc_rows_dist.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                    ctypes.c_int32, _i64p, ctypes.c_int64,
                                    _f64p]
        L.orc_tree_build.restype = ctypes.c_int64
        L.orc_tree_build.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_int32,
                                     _i32p, _i32p, _f64p, _i32p, _i32p,
                                     _i32p, _i32p, _i32p]
        L.orc_tree_query.restype = ctypes.c_int64
        L.orc_tree_query.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                     ctypes.c_int32, ctypes.c_double,
                                     _i32p, _i32p, _f64p, _i32p, _i32p,
                                     _i32p, _i32p, ctypes.c_int64, _i64p,
                                     _vp, _vp]
        L.orc_check_tree.restype = None
        L.orc_check_tree.argtypes = [ctypes.c_int, _vp, ctypes.c_int64,
                                     ctypes.c_int32, _i32p, _i32p, _f64p,
                                     _i32p, _i32p, _i32p, _i32p, _i32p,
                                     ctypes.c_int64, _i64p]
        _lib = L
    return _lib


def _prep(points: np.ndarray, metric: int):
    """Contiguous buffer and the library's ``dim`` for a point array."""
    if metric in (L2, ANGULAR):
        a = np.ascontiguousarray(points, dtype=np.float32)
        return a, a.shape[0], a.shape[1]
    if metric == HAMMING:
        a = np.ascontiguousarray(points, dtype=np.uint64)
        return a, a.shape[0], a.shape[1] * 64
    a = np.ascontiguousarray(points, dtype=np.uint8)
    return a, a.shape[0], a.shape[1]


def eps_param(metric: int, eps: float) -> float:
    return lib().orc_eps_param(metric, float(eps))


# ---- pair primitives -------------------------------------------------------

def l2_sq(x, y) -> float:
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    return lib().orc_l2_sq(x, y, x.size)


def ang_terms(x, y):
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    g, a, b = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().orc_ang_terms(x, y, x.size, ctypes.byref(g), ctypes.byref(a),
                        ctypes.byref(b))
    return g.value, a.value, b.value


def ang_pred(g, a, b, C) -> bool:
    return bool(lib().orc_ang_pred(g, a, b, C))


def ang_dist(x, y) -> float:
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    return lib().orc_ang_dist(x, y, x.size)


def ham(x, y) -> int:
    x = np.ascontiguousarray(x, np.uint64)
    y = np.ascontiguousarray(y, np.uint64)
    return lib().orc_ham(x, y, x.size)


def _as_str(s) -> np.ndarray:
    """uint8 symbols of a string given as bytes/list/array; a padded row is
    cut at its first 0xFF.  Never empty as a buffer (length passed apart)."""
    if isinstance(s, (bytes, bytearray, list, tuple)):
        a = np.asarray(list(s), dtype=np.uint8)
    else:
        a = np.asarray(s, dtype=np.uint8).ravel()
    pad = np.nonzero(a == 0xFF)[0]
    if pad.size:
        a = a[:pad[0]]
    return a


def _buf(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a) if a.size else np.zeros(1, np.uint8)


def lev(a, b) -> int:
    """Unit-cost edit distance (Wagner-Fischer)."""
    a, b = _as_str(a), _as_str(b)
    return lib().orc_lev(_buf(a), int(a.size), _buf(b), int(b.size))


def lev_banded(a, b, k: int) -> int:
    """min(lev(a, b), k + 1) from the band |i - j| <= k."""
    a, b = _as_str(a), _as_str(b)
    return lib().orc_lev_banded(_buf(a), int(a.size), _buf(b), int(b.size),
                                int(k))


# ---- the epsilon-graph -----------------------------------------------------

def bruteforce(points: np.ndarray, metric: int, eps: float, rows=None):
    """Ordered-pair epsilon-graph by exhaustive pinned predicate.

    Returns (row_ptr int64 [R+1], col int32 [nnz], dist float64 [nnz]) with
    columns ascending.  ``rows`` restricts to the listed rows (in that
    order) against all points."""
    a, n, dim = _prep(points, metric)
    L = lib()
    if rows is None:
        rp, R = None, n
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        rp, R = rows.ctypes.data, rows.size
    deg = np.zeros(max(R, 1), dtype=np.int64)
    total = L.orc_bf_count(metric, a.ctypes.data, n, dim, float(eps), rp, R,
                           deg)
    row_ptr = np.zeros(R + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(deg[:R])
    col = np.zeros(max(total, 1), dtype=np.int32)
    dist = np.zeros(max(total, 1), dtype=np.float64)
    L.orc_bf_fill(metric, a.ctypes.data, n, dim, float(eps), rp, R, row_ptr,
                  col, dist)
    return row_ptr, col[:total], dist[:total]


def rows_dist(points: np.ndarray, metric: int, rows) -> np.ndarray:
    """FP64 distances from the listed rows to every point [len(rows), n]."""
    a, n, dim = _prep(points, metric)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty((rows.size, n), dtype=np.float64)
    lib().orc_rows_dist(metric, a.ctypes.data, n, dim, rows, rows.size, out)
    return out


def tree_build(points: np.ndarray, metric: int, zeta: int = 1) -> dict:
    """Batch cover tree (Algorithms 1-2).  Arrays follow the layout described
    in fnn_oracle.c."""
    a, n, dim = _prep(points, metric)
    cap = 2 * n + 1
    order = np.zeros(n, np.int32)
    center = np.zeros(cap, np.int32)
    radius = np.zeros(cap, np.float64)
    level = np.zeros(cap, np.int32)
    cb = np.zeros(cap, np.int32)
    cc = np.zeros(cap, np.int32)
    pb = np.zeros(cap, np.int32)
    pe = np.zeros(cap, np.int32)
    nn = lib().orc_tree_build(metric, a.ctypes.data, n, dim, int(zeta), order,
                              center, radius, level, cb, cc, pb, pe)
    if nn < 0:
        raise ValueError("oracle tree build rejected its input")
    return dict(order=order, center=center[:nn].copy(),
                radius=radius[:nn].copy(), level=level[:nn].copy(),
                child_begin=cb[:nn].copy(), child_count=cc[:nn].copy(),
                pt_begin=pb[:nn].copy(), pt_end=pe[:nn].copy(), nnodes=nn)


def tree_query(points: np.ndarray, metric: int, eps: float, tree: dict):
    """All-points range query through the tree (Algorithm 3)."""
    a, n, dim = _prep(points, metric)
    L = lib()
    t = {k: np.ascontiguousarray(v) for k, v in tree.items()
         if isinstance(v, np.ndarray)}
    row_ptr = np.zeros(n + 1, np.int64)
    args = (metric, a.ctypes.data, n, dim, float(eps), t["order"], t["center"],
            np.ascontiguousarray(t["radius"], np.float64), t["child_begin"],
            t["child_count"], t["pt_begin"], t["pt_end"], int(tree["nnodes"]),
            row_ptr)
    total = L.orc_tree_query(*args, None, None)
    col = np.zeros(max(total, 1), np.int32)
    dist = np.zeros(max(total, 1), np.float64)
    L.orc_tree_query(*args, col.ctypes.data, dist.ctypes.data)
    return row_ptr, col[:total], dist[:total]


INVARIANTS = ("I1_partition", "I2_nesting", "I3a_child_covering",
              "I3b_radius", "I3c_split_covering", "I4_separation",
              "I5_levels", "structure")


def check_tree(points: np.ndarray, metric: int, tree: dict) -> dict:
    """Counts of cover-tree invariant violations (all zero for a valid tree)."""
    a, n, dim = _prep(points, metric)
    viol = np.zeros(8, np.int64)
    lib().orc_check_tree(
        metric, a.ctypes.data, n, dim,
        np.ascontiguousarray(tree["order"], np.int32),
        np.ascontiguousarray(tree["center"], np.int32),
        np.ascontiguousarray(tree["radius"], np.float64),
        np.ascontiguousarray(tree["level"], np.int32),
        np.ascontiguousarray(tree["child_begin"], np.int32),
        np.ascontiguousarray(tree["child_count"], np.int32),
        np.ascontiguousarray(tree["pt_begin"], np.int32),
        np.ascontiguousarray(tree["pt_end"], np.int32),
        int(tree["nnodes"]), viol)
    return dict(zip(INVARIANTS, (int(v) for v in viol)))


# ---- CSR comparison ----------------------------------------------------------

def compare_csr(row_ptr, col, dist, ref_row_ptr, ref_col, ref_dist,
                rtol: float = 1e-5, atol: float = 0.0) -> dict:
    """Edge-set and distance comparison of a candidate CSR against the
    oracle's.  Edge sets must be identical (row_ptr and col equal); distances
    within rtol relative (plus atol absolute) of the FP64 value."""
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    ref_row_ptr = np.asarray(ref_row_ptr, np.int64)
    ref_col = np.asarray(ref_col, np.int64)
    out = dict(rows=int(ref_row_ptr.size - 1), nnz=int(col.size),
               ref_nnz=int(ref_col.size))
    out["row_ptr_equal"] = bool(row_ptr.shape == ref_row_ptr.shape and
                                np.array_equal(row_ptr, ref_row_ptr))
    if out["row_ptr_equal"] and col.size == ref_col.size:
        out["col_equal"] = bool(np.array_equal(col, ref_col))
    else:
        out["col_equal"] = False
    # missing / extra edges, counted as sets of (row, col)
    R = ref_row_ptr.size - 1
    rr = np.repeat(np.arange(R, dtype=np.int64), np.diff(ref_row_ptr))
    cr = np.repeat(np.arange(row_ptr.size - 1, dtype=np.int64), np.diff(row_ptr))
    ka = cr * (1 << 32) + col
    kb = rr * (1 << 32) + ref_col
    out["extra"] = int(np.setdiff1d(ka, kb).size)
    out["missing"] = int(np.setdiff1d(kb, ka).size)
    if out["col_equal"]:
        d = np.asarray(dist, np.float64)
        r = np.asarray(ref_dist, np.float64)
        err = np.abs(d - r)
        lim = rtol * np.abs(r) + atol
        out["max_rel_err"] = float(np.max(err / np.maximum(np.abs(r), 1e-300))) if r.size else 0.0
        out["max_abs_err"] = float(err.max()) if r.size else 0.0
        out["dist_ok"] = bool(np.all(err <= lim))
    else:
        out["dist_ok"] = False
    out["ok"] = out["row_ptr_equal"] and out["col_equal"] and out["dist_ok"]
    return out


def csr_symmetric(row_ptr, col, dist=None) -> bool:
    """j in row i <=> i in row j (with identical distance bits), no self
    loops, columns strictly ascending within each row."""
    row_ptr = np.asarray(row_ptr, np.int64)
    col = np.asarray(col, np.int64)
    n = row_ptr.size - 1
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    if np.any(rows == col):
        return False
    # strictly ascending within rows
    if col.size > 1:
        same = rows[1:] == rows[:-1]
        if np.any(col[1:][same] <= col[:-1][same]):
            return False
    fwd = rows * n + col
    bwd = col * n + rows
    o1 = np.argsort(fwd, kind="stable")
    o2 = np.argsort(bwd, kind="stable")
    if not np.array_equal(fwd[o1], bwd[o2]):
        return False
    if dist is not None:
        d = np.asarray(dist)
        if not np.array_equal(d[o1].view(np.uint8), d[o2].view(np.uint8)):
            return False
    return True
