"""The C-ABI library loads and exports every symbol include/fnn.h declares;
argument checks that need no GPU (CPU only, no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fnn.h")
LIB = os.path.join(ROOT, "paper_2510_14147_amd", "libfnn.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fnn_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2510_14147_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert "fnn_tree_build" in names and "fnn_eps_graph" in names
    assert "fnn_free" in names
    for n in names:
        assert hasattr(lib, n), n


def test_version_and_error_string(lib):
    lib.fnn_version.restype = ctypes.c_int
    assert lib.fnn_version() >= 100
    lib.fnn_last_error.restype = ctypes.c_char_p
    assert isinstance(lib.fnn_last_error(), bytes)


def test_argument_errors_without_gpu(lib):
    vp = ctypes.c_void_p
    out = vp(123)
    lib.fnn_tree_build.argtypes = [vp, ctypes.c_int64, ctypes.c_int32,
                                   ctypes.c_int, ctypes.POINTER(vp)]
    assert lib.fnn_tree_build(None, 10, 4, 0, ctypes.byref(out)) == -1
    assert out.value is None
    lib.fnn_last_error.restype = ctypes.c_char_p
    assert b"NULL" in lib.fnn_last_error()
    assert lib.fnn_tree_build(vp(16), 0, 4, 0, ctypes.byref(out)) == -1
    assert lib.fnn_tree_build(vp(16), 10, 4, 7, ctypes.byref(out)) == -1
    lib.fnn_eps_graph.argtypes = [vp, ctypes.c_double, ctypes.POINTER(vp)]
    assert lib.fnn_eps_graph(None, 1.0, ctypes.byref(out)) == -1
    lib.fnn_free.argtypes = [vp]
    lib.fnn_free(None)
    # batch of clouds: offsets are checked on the host before any device work
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.fnn_tree_build_batch.argtypes = [vp, i64p, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int, vp, ctypes.POINTER(vp)]

    def offs(*v):
        return (ctypes.c_int64 * len(v))(*v)

    assert lib.fnn_tree_build_batch(vp(16), None, 2, 4, 0, None, ctypes.byref(out)) == -1
    assert b"offsets" in lib.fnn_last_error()
    assert lib.fnn_tree_build_batch(vp(16), offs(0, 5), 0, 4, 0, None,
                                    ctypes.byref(out)) == -1
    assert lib.fnn_tree_build_batch(vp(16), offs(1, 5, 9), 2, 4, 0, None,
                                    ctypes.byref(out)) == -1
    assert lib.fnn_tree_build_batch(vp(16), offs(0, 7, 5, 9), 3, 4, 0, None,
                                    ctypes.byref(out)) == -1
    assert b"non-decreasing" in lib.fnn_last_error()
    assert lib.fnn_tree_build_batch(vp(16), offs(0, 0, 0), 2, 4, 0, None,
                                    ctypes.byref(out)) == -1  # every cloud empty
    assert lib.fnn_tree_build_batch(None, offs(0, 3), 1, 4, 0, None,
                                    ctypes.byref(out)) == -1
    assert out.value is None
    lib.fnn_eps_graph_batch.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.c_int32, vp, ctypes.POINTER(vp)]
    e2 = (ctypes.c_double * 2)(1.0, 2.0)
    assert lib.fnn_eps_graph_batch(None, e2, 2, None, ctypes.byref(out)) == -1
    lib.fnn_autotune.argtypes = [vp, i64p, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_double), vp,
                                 ctypes.c_int32, vp]
    res = ctypes.create_string_buffer(256)
    assert lib.fnn_autotune(vp(16), None, 1, 4, 0, e2, None, 1, res) == -1
    assert lib.fnn_autotune(vp(16), offs(3, 9), 1, 4, 0, e2, None, 1, res) == -1
    assert b"offsets" in lib.fnn_last_error()
    lib.fnn_set_allocator.argtypes = [vp, vp, vp]
    assert lib.fnn_set_allocator(vp(1), None, None) == -1
    # bichromatic query: the tree handle and out are checked first
    lib.fnn_eps_query.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, vp,
                                  ctypes.POINTER(vp)]
    out = vp(123)
    assert lib.fnn_eps_query(None, vp(16), 4, 1.0, None, ctypes.byref(out)) == -1
    assert out.value is None
    assert b"tree" in lib.fnn_last_error()
    assert lib.fnn_eps_query(None, vp(16), 4, 1.0, None, None) == -1


def _header_fields(struct):
    import re
    h = open(os.path.join(ROOT, "include", "fnn.h")).read()
    body = h[h.index("typedef struct %s {" % struct):]
    body = body[:body.index("}")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split("{", 1)[1].split(";"):
        decl = decl.strip()
        if not decl:
            continue
        for part in decl.split(","):
            nm = re.findall(r"(\w+)\s*(?:\[\d+\])?\s*$", part.strip())
            names.append(nm[0])
    return names


def test_options_struct_matches_header():
    from paper_2510_14147_amd import fnn_options, fnn_stats, fnn_csr
    assert [f[0] for f in fnn_options._fields_] == _header_fields("fnn_options")
    assert [f[0] for f in fnn_stats._fields_] == _header_fields("fnn_stats")
    assert ctypes.sizeof(fnn_options) == 16 * 4
    from paper_2510_14147_amd import fnn_tune_result
    assert [f[0] for f in fnn_tune_result._fields_] == _header_fields("fnn_tune_result")
    assert ctypes.sizeof(fnn_tune_result) == 64 + 8 + 8 + 4 + 4 + 4 * 8
    assert ctypes.sizeof(fnn_csr) == 8 + 8 + 8 + 3 * 8
    assert ctypes.sizeof(fnn_stats) == 17 * 8 + 12 * 8 + 8 + 8 + 8 + 5 * 8 + 3 * 8 + 8


def test_alloc_callback_reports_failure_as_null():
    """The Python allocator behind fnn_set_allocator must hand the library a
    NULL (which it turns into FNN_ENOMEM) when torch cannot allocate: an
    exception escaping a ctypes callback would leave an undefined pointer."""
    import ctypes
    import paper_2510_14147_amd as f
    call = f._ALLOC_FN(ctypes.cast(f._alloc_cb, ctypes.c_void_p).value)
    for _ in range(3):
        assert call(1 << 62, None) in (None, 0)
