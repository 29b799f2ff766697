"""The allocation-free gradient entry point (GPU): fnn_mlp_loss_grad_noalloc
called through the C ABI against fnn_mlp_loss_grad on the same inputs, on two
calls in a row (the second with fewer samples, so stale partial rows of the
first call must not leak into it), plus bit-identical repeats."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fnn():
    import torch
    assert torch.cuda.is_available()
    import paper_2510_14147_amd as f
    f.lib()
    return f


def _inputs(seed, n):
    import torch
    from oracle import mlp
    rng = np.random.default_rng(seed)
    th = mlp.init(seed).astype(np.float32)
    th[-2:] = rng.normal(0, 0.3, 2)
    x = rng.normal(0, 1, (n, 16)).astype(np.float32)
    t = rng.normal(0, 1, (n, 2)).astype(np.float32)
    return (torch.from_numpy(th).cuda(), torch.from_numpy(x).cuda(),
            torch.from_numpy(t).cuda())


def _noalloc(fnn, th, X, T):
    """Direct C-ABI call with caller-owned device outputs."""
    import torch
    L = fnn.lib()
    g = torch.full((fnn.MLP_NPARAMS,), float("nan"), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    fnn._bind_stream()
    rc = L.fnn_mlp_loss_grad_noalloc(ctypes.c_void_p(th.data_ptr()),
                                     ctypes.c_void_p(X.data_ptr()),
                                     ctypes.c_void_p(T.data_ptr()), X.shape[0],
                                     ctypes.c_void_p(g.data_ptr()),
                                     ctypes.c_void_p(loss.data_ptr()))
    assert rc == 0, L.fnn_last_error()
    torch.cuda.synchronize()
    return float(loss.item()), g.cpu().numpy()


def _check(fnn, th, X, T):
    l_ref, g_ref = fnn.fnn_mlp_loss_grad(th, X, T)
    g_ref = g_ref.cpu().numpy()
    l, g = _noalloc(fnn, th, X, T)
    assert abs(l - l_ref) <= 1e-6 * abs(l_ref), (l, l_ref)
    scale = np.abs(g_ref).max()
    # the two sum the same FP32 products in different orders (atomics vs a
    # fixed tree): agreement to FP32 summation error
    np.testing.assert_allclose(g, g_ref, rtol=1e-4, atol=1e-5 * scale)
    return l, g


def test_noalloc_matches_allocating_entry_point_twice(fnn):
    print("[case] noalloc grad n=70000 then n=1000", flush=True)
    th, X, T = _inputs(4, 70_000)      # uses all 256 partial rows
    l1, g1 = _check(fnn, th, X, T)
    th2, X2, T2 = _inputs(5, 1000)     # 32 rows: the other rows hold call 1
    l2, g2 = _check(fnn, th2, X2, T2)
    assert l1 != l2
    # repeats give identical bits (fixed summation order, no atomics)
    l3, g3 = _noalloc(fnn, th2, X2, T2)
    assert l3 == l2 and np.array_equal(g3.view(np.uint32), g2.view(np.uint32))


def test_noalloc_small_and_empty(fnn):
    import torch
    print("[case] noalloc grad n=1, n=0", flush=True)
    th, X, T = _inputs(6, 1)
    _check(fnn, th, X, T)
    l, g = _noalloc(fnn, th, X[:0], T[:0])
    assert l == 0.0 and not np.any(g)


def test_noalloc_argument_errors(fnn):
    L = fnn.lib()
    vp = ctypes.c_void_p
    assert L.fnn_mlp_loss_grad_noalloc(None, vp(16), vp(16), 4, vp(16), vp(16)) == -1
    assert L.fnn_mlp_loss_grad_noalloc(vp(16), vp(16), vp(16), 4, vp(16), None) == -1
    assert L.fnn_mlp_loss_grad_noalloc(vp(16), vp(16), vp(16), (1 << 31) + 1,
                                       vp(16), vp(16)) == -1
    assert b"FNN_NOALLOC_MAX_SAMPLES" in L.fnn_last_error()
