"""GPU parity of the products with coupling matrices evaluated on the fly
(recompute_coupling): S_ts = g(xi_t, xi_s) at the interpolation points is
the same matrix as the stored one, so the product equals the oracle's dense
H^2 matrix to rounding, for one vector and for blocks of right-hand sides,
A x and A^T x, orders 2 to 6 (k = 8 ... 216 coefficients per cluster, more
than one wave of rows from order 5 on).  After recompression the projections
onto the interpolation bases are applied per cluster; the product equals the
stored recompressed operator's to rounding."""
import numpy as np
import pytest

import oracle
import synth
from oracle import h2

pytestmark = pytest.mark.gpu

_dense_cache = {}


def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2001_05523_amd as h
    return h


def _dense(s, kernel, q=4):
    key = (s, kernel, q)
    if key not in _dense_cache:
        v, t = synth.octa_sphere(s)
        _dense_cache[key] = (oracle.slp_dense if kernel == "slp" else oracle.dlp_dense)(v, t, q)
    return _dense_cache[key]


def _run(op, X, trans=False, alpha=1.0):
    import torch
    nout = op.shape[1] if trans else op.shape[0]
    if X.ndim == 1:
        Xd = torch.tensor(X, device="cuda")
        Yd = torch.zeros(nout, dtype=torch.float64, device="cuda")
    else:
        Xd = torch.tensor(np.asfortranarray(X), device="cuda").t().contiguous().t()
        Yd = torch.zeros((X.shape[1], nout), dtype=torch.float64, device="cuda").t()
    op.matvec(Xd, Yd, alpha=alpha, trans=trans)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("kernel,s,leaf,m", [("slp", 8, 16, 2), ("slp", 8, 16, 3), ("dlp", 8, 16, 3),
                                             ("slp", 16, 32, 4), ("dlp", 16, 32, 4), ("slp", 8, 8, 5),
                                             ("dlp", 8, 8, 6)])
def test_evaluated_coupling_against_oracle_h2(kernel, s, leaf, m):
    h = _lib()
    v, t = synth.octa_sphere(s)
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=4, recompute_coupling=True)
    info = op.info()
    assert info["nfar"] > 0 and info["coupling_entries"] == 0
    assert info["coupling_evals"] == info["nfar"] * m ** 6
    A = _dense(s, kernel)
    H, _ = h2.h2_dense(v, t, kernel, leaf, m, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        for nrhs in (1, 16, 64):
            X = synth.random_vector(nin, 451 + trans, cols=None if nrhs == 1 else nrhs)
            Y = _run(op, X, trans=trans, alpha=0.75)
            ref = 0.75 * ((H.T if trans else H) @ X)
            d = np.max(np.abs(Y - ref)) / np.max(np.abs(ref))
            print("%s m=%d trans=%d nrhs=%d: max rel diff %.2e" % (kernel, m, trans, nrhs, d))
            assert d <= 1e-11, (trans, nrhs, d)


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_evaluated_coupling_after_recompression(kernel):
    """Recompressed order-4 bases (1e-6): the evaluated coupling with the
    per-cluster projections equals the stored recompressed coupling to
    rounding, and both stay within 20 x 1e-6 of the oracle's H^2 matrix; the
    operator stores no coupling matrices."""
    h = _lib()
    s, leaf = 16, 16
    v, t = synth.octa_sphere(s)
    kw = dict(kernel=kernel, leaf=leaf, order_m=4, q_near=4, recompress_tol=1e-6)
    stored = h.Operator(v, t, **kw)
    evald = h.Operator(v, t, recompute_coupling=True, **kw)
    i_s, i_e = stored.info(), evald.info()
    assert i_e["coupling_entries"] == 0 and i_s["coupling_entries"] > 0
    assert i_e["mean_rank_row"] == i_s["mean_rank_row"]
    A = _dense(s, kernel)
    H, _ = h2.h2_dense(v, t, kernel, leaf, 4, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        for nrhs in (1, 32):
            X = synth.random_vector(nin, 461 + trans, cols=None if nrhs == 1 else nrhs)
            ys, ye = _run(stored, X, trans=trans), _run(evald, X, trans=trans)
            d = np.max(np.abs(ye - ys)) / np.max(np.abs(ys))
            ref = (H.T if trans else H) @ X
            err = np.linalg.norm(ye - ref) / np.linalg.norm(ref)
            print("%s trans=%d nrhs=%d: evaluated vs stored %.2e, vs oracle H2 %.2e" % (kernel, trans, nrhs, d, err))
            assert d <= 1e-12, d
            assert err <= 20e-6, err


def test_evaluated_coupling_requests_refused():
    """Evaluated couplings need an FP64 interpolation far field."""
    h = _lib()
    v, t = synth.octa_sphere(4)
    for kw in (dict(farfield_dtype="f32", recompress_tol=1e-6), dict(farfield_dtype="bf16", recompress_tol=1e-6),
               dict(gca_tol=1e-4)):
        with pytest.raises(h.H2BError) as e:
            h.Operator(v, t, kernel="slp", leaf=8, order_m=3, q_near=4, recompute_coupling=True, **kw)
        assert e.value.code == h.H2B_ENOTSUP, kw


def test_evaluated_coupling_shape_gradient_and_tuning():
    """The shape gradient and the block-width tuner run on evaluated couplings
    and agree with the stored-coupling operator."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(8)
    a = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4)
    b = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4, recompute_coupling=True)
    x = torch.tensor(synth.random_vector(len(t), 471), device="cuda")
    y = torch.tensor(synth.random_vector(len(t), 472), device="cuda")
    ga, gb = a.shape_grad(x, y), b.shape_grad(x, y)
    torch.cuda.synchronize()
    assert float((ga - gb).abs().max()) <= 1e-12 * float(ga.abs().max())
    assert b.tune(64) > 0
    X = synth.random_vector(len(t), 473, cols=64)
    Ya, Yb = _run(a, X), _run(b, X)
    assert np.max(np.abs(Ya - Yb)) <= 1e-12 * np.max(np.abs(Ya))
