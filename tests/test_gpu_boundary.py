"""GPU checks of the C-ABI boundary: the installed device allocator and the
single-layer bilinear form."""
import gc

import numpy as np
import pytest

import oracle
import synth
from oracle import h2

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2001_05523_amd as h
    return h


def test_operator_memory_comes_from_torch_allocator():
    """With torch's caching allocator installed (the binding's default) the
    operator's device bytes show in torch.cuda.memory_allocated() and go back
    when it is destroyed; with hipMalloc they do not show."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(16)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    op = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
    info = op.info()
    grown = torch.cuda.memory_allocated() - base
    stored = info["bytes_near"] + info["bytes_far"] + info["bytes_transposed"] + info["bytes_vectors"]
    print("torch sees %d bytes for %d stored" % (grown, stored))
    assert grown >= stored
    x = torch.tensor(synth.random_vector(op.shape[1], 5), device="cuda")
    y = torch.zeros(op.shape[0], dtype=torch.float64, device="cuda")
    op.matvec(x, y)
    torch.cuda.synchronize()
    del op
    gc.collect()
    assert torch.cuda.memory_allocated() - base <= 2 * 1024 * 1024  # x and y
    try:
        h.use_hip_allocator()
        base = torch.cuda.memory_allocated()
        op = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
        assert torch.cuda.memory_allocated() == base
        y2 = torch.zeros_like(y)
        op.matvec(x, y2)
        torch.cuda.synchronize()
        assert torch.equal(y, y2)
        del op
        gc.collect()
    finally:
        h.use_torch_allocator()


def test_slp_bilinear_against_oracle():
    """x^T G y through h2b_slp_bilinear equals x^T H y with the oracle's dense
    H^2 matrix H to rounding; gy equals H y."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4)
    A = oracle.slp_dense(v, t, 4)
    H, _ = h2.h2_dense(v, t, "slp", 16, 3, near_matrix=A)
    x, y = synth.random_vector(len(t), 61), synth.random_vector(len(t), 62)
    X = torch.tensor(x, device="cuda")
    Y = torch.tensor(y, device="cuda")
    GY = torch.full_like(X, 7.0)  # overwritten
    b = torch.zeros((), dtype=torch.float64, device="cuda")
    h._check(h.h2b_slp_bilinear(op.handle, h._vp(X.data_ptr()), h._vp(Y.data_ptr()), h._vp(GY.data_ptr()),
                                h._vp(b.data_ptr()), None))
    torch.cuda.synchronize()
    ref = H @ y
    assert np.max(np.abs(GY.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert abs(float(b) - x @ ref) <= 1e-12 * np.abs(x).dot(np.abs(ref))
    with pytest.raises(h.H2BError):
        h._check(h.h2b_slp_bilinear(op.handle, h._vp(X.data_ptr()), h._vp(Y.data_ptr()), h._vp(X.data_ptr()),
                                    h._vp(b.data_ptr()), None))


def test_matmul_operator_and_transpose():
    """op @ x and op.T @ x (the binding's product notation) equal the
    library's products, for a vector and for a block of right-hand sides
    given row-major (the binding makes its columns contiguous)."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(8)
    K = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
    x = torch.tensor(synth.random_vector(K.shape[1], 71), device="cuda")
    y = torch.zeros(K.shape[0], dtype=torch.float64, device="cuda")
    K.matvec(x, y)
    assert torch.equal(K @ x, y)
    w = torch.tensor(synth.random_vector(K.shape[0], 72), device="cuda")
    z = torch.zeros(K.shape[1], dtype=torch.float64, device="cuda")
    K.matvec(w, z, trans=True)
    assert torch.equal(K.T @ w, z) and K.T.shape == (K.shape[1], K.shape[0])
    X = torch.tensor(synth.random_vector(K.shape[1], 73, cols=5), device="cuda")  # row-major
    Y = K @ X
    assert Y.shape == (K.shape[0], 5)
    for c in range(5):
        yc = torch.zeros(K.shape[0], dtype=torch.float64, device="cuda")
        K.matvec(X[:, c].contiguous(), yc)
        assert float((Y[:, c] - yc).abs().max()) <= 1e-12 * float(yc.abs().max())
