"""The allocation-free product h2b_matvec_noalloc (work vectors in the
library's static device array) against h2b_matvec, through the C ABI: two
calls in a row, the second with a smaller input, both equal to the ordinary
product to rounding; no device allocation happens during the calls; requests
beyond the array are refused before any launch."""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2001_05523_amd as h
    return h


def _cols(torch, a):
    return torch.tensor(np.asfortranarray(a), device="cuda").t().contiguous().t() if a.ndim == 2 else \
        torch.tensor(a, device="cuda")


def _call(h, fn, op, X, Y, trans, alpha):
    nrhs = 1 if X.dim() == 1 else X.shape[1]
    ldx = X.shape[0] if X.dim() == 1 else X.stride(1)
    ldy = Y.shape[0] if Y.dim() == 1 else Y.stride(1)
    h._check(fn(op.handle, int(trans), float(alpha), h._vp(X.data_ptr()), ldx, h._vp(Y.data_ptr()), ldy, nrhs,
                None))


def test_noalloc_product_matches_matvec_twice():
    import torch
    h = _lib()
    cases = []
    # first call: K on 2,048 triangles with 16 right-hand sides, transposed;
    # second call: G on 512 triangles, one vector (smaller work vectors, so
    # stale contents of the first call stay behind in the array)
    v1, t1 = synth.octa_sphere(16)
    op1 = h.Operator(v1, t1, kernel="dlp", leaf=16, order_m=3, q_near=4)
    cases.append((op1, True, 16, 0.5, 401))
    v2, t2 = synth.octa_sphere(8)
    op2 = h.Operator(v2, t2, kernel="slp", leaf=16, order_m=3, q_near=4)
    cases.append((op2, False, 1, -1.25, 402))
    calls = []

    def alloc(nbytes, stream, ctx):
        calls.append(nbytes)
        return None

    def free(ptr, stream, ctx):
        calls.append(-1)

    a, f = h._ALLOC_FN(alloc), h._FREE_FN(free)
    for op, trans, nrhs, alpha, seed in cases:
        nin = op.shape[0] if trans else op.shape[1]
        nout = op.shape[1] if trans else op.shape[0]
        X = _cols(torch, synth.random_vector(nin, seed, cols=None if nrhs == 1 else nrhs))
        y0 = synth.random_vector(nout, seed + 1, cols=None if nrhs == 1 else nrhs)
        Y_ref, Y = _cols(torch, y0), _cols(torch, y0)
        _call(h, h.h2b_matvec, op, X, Y_ref, trans, alpha)
        torch.cuda.synchronize()
        # any device allocation inside the call would reach this allocator
        h._check(h.h2b_set_allocator(a, f, None))
        try:
            _call(h, h.h2b_matvec_noalloc, op, X, Y, trans, alpha)
            torch.cuda.synchronize()
        finally:
            h.use_torch_allocator()
        assert calls == []
        ref = Y_ref.cpu().numpy()
        got = Y.cpu().numpy()
        scale = np.max(np.abs(ref - y0))
        print("trans=%d nrhs=%d: max diff %.2e of %.2e" % (trans, nrhs, np.max(np.abs(got - ref)), scale))
        assert np.max(np.abs(got - ref)) <= 1e-12 * scale


def test_noalloc_refuses_work_beyond_the_array():
    """64 right-hand sides on 131,072 triangles need 3 x 131,072 x 64 doubles
    of vectors alone (201 MB), more than the 128 MiB array: refused with
    H2B_EINVAL before any launch, y untouched."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(128)
    op = h.Operator(v, t, kernel="slp", leaf=64, order_m=2, q_near=2)
    X = torch.ones((64, len(t)), dtype=torch.float64, device="cuda").t()
    Y = torch.full((64, len(t)), 3.0, dtype=torch.float64, device="cuda").t()
    rc = h.h2b_matvec_noalloc(op.handle, 0, 1.0, h._vp(X.data_ptr()), len(t), h._vp(Y.data_ptr()), len(t), 64,
                              None)
    assert rc == h.H2B_EINVAL
    assert b"static scratch" in h.h2b_last_error()
    torch.cuda.synchronize()
    assert bool(torch.all(Y == 3.0))
