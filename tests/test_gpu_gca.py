"""GPU parity of the Green cross approximation (Section 4) of the single-layer
matrix G and the double-layer matrix K: the HIP product of the GCA H^2 matrix
against the oracle's dense GCA matrix (same trees, same boxes, same
quadrature, same pivoting rule) and against the dense Galerkin matrix."""
import numpy as np
import pytest

import oracle
import synth
from oracle import gca

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _lib():
    import paper_2001_05523_amd as h
    return h


def _product(op, x, trans=False):
    torch = _torch()
    X = torch.tensor(x, dtype=torch.float64, device="cuda")
    Y = torch.zeros(op.shape[0], dtype=torch.float64, device="cuda")
    op.matvec(X, Y, trans=trans)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("m,eps", [(2, 1e-2), (3, 1e-4), (4, 1e-6)])
def test_gca_product_matches_oracle_gca(m, eps):
    """On a perturbed sphere (no mirror symmetries, so no ties in the
    pivoting) the library picks the oracle's pivots: same ranks, and the
    products G x and G^T x equal the oracle's dense GCA matrix to rounding
    (1e-10)."""
    h = _lib()
    v, t = synth.perturbed_sphere(8, seed=3)
    G = oracle.slp_dense(v, t, 4)
    A, info = gca.gca_dense(v, t, 16, m, eps, G)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=m, q_near=4, gca_tol=eps)
    st = op.info()
    ranks = np.array(list(info["ranks"].values()))
    assert st["row_coeffs"] == ranks.sum() and st["max_rank_row"] == ranks.max()
    for trans in (False, True):
        x = synth.random_vector(len(t), 71 + trans)
        y = _product(op, x, trans)
        assert _rel(y, (A.T if trans else A) @ x) <= 1e-10, (m, eps, trans)


def test_gca_once_per_pair_coupling_matches_full():
    """The cross approximation's couplings of G are entries between pivot
    triangles of admissible clusters, symmetric to rounding, so G's far field
    is stored once per pair (half the coupling entries, ranks above 64
    included) and G x, G^T x equal the products from the full panels to
    rounding."""
    h = _lib()
    v, t = synth.perturbed_sphere(16, seed=5)
    kw = dict(kernel="slp", leaf=16, order_m=4, q_near=4, gca_tol=1e-8)
    a = h.Operator(v, t, symmetric_near=True, **kw)
    b = h.Operator(v, t, symmetric_near=False, **kw)
    ia, ib = a.info(), b.info()
    assert ia["max_rank_row"] > 64
    assert ib["cpl_sym_entries"] == 0 and 2 * ia["cpl_sym_entries"] == ia["coupling_entries"]
    for trans in (False, True):
        x = synth.random_vector(len(t), 81 + trans)
        ya, yb = _product(a, x, trans), _product(b, x, trans)
        assert float(np.max(np.abs(ya - yb)) / np.max(np.abs(yb))) <= 1e-13, trans


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_gca_recompressed_against_oracle_gca(kernel):
    """Algebraic recompression (Section 5) of the cross-approximation bases,
    whose ranks reach 176 here (the tiled sandwich and Gram kernels): the
    products stay within a small multiple of the tolerance of the oracle's
    dense GCA matrix, with fewer coefficients and coupling entries."""
    torch = _torch()
    h = _lib()
    v, t = synth.perturbed_sphere(16, seed=5)
    eps, tol = 1e-8, 1e-6
    if kernel == "slp":
        A, _ = gca.gca_dense(v, t, 16, 4, eps, oracle.slp_dense(v, t, 4))
    else:
        A, _ = gca.gca_dense_dlp(v, t, 16, 4, eps, oracle.dlp_dense(v, t, 4))
    kw = dict(kernel=kernel, leaf=16, order_m=4, q_near=4, gca_tol=eps)
    plain = h.Operator(v, t, **kw)
    rc = h.Operator(v, t, recompress_tol=tol, **kw)
    ip, ir = plain.info(), rc.info()
    assert ip["max_rank_row"] > 64
    assert ir["row_coeffs"] < ip["row_coeffs"] and ir["coupling_entries"] < ip["coupling_entries"]
    for trans in (False, True):
        x = synth.random_vector(A.shape[0] if trans else A.shape[1], 91 + trans)
        X = torch.tensor(x, device="cuda")
        y = ((rc.T if trans else rc) @ X).cpu().numpy()
        ref = (A.T if trans else A) @ x
        err = _rel(y, ref)
        print("%s trans=%d recompressed GCA vs oracle GCA: %.3e, coefficients %d -> %d"
              % (kernel, trans, err, ip["row_coeffs"], ir["row_coeffs"]))
        assert err <= 20 * tol


@pytest.mark.parametrize("m,eps", [(2, 1e-2), (3, 1e-4)])
def test_gca_double_layer_matches_oracle_gca(m, eps):
    """K: triangle rows with the bases of G, vertex columns from the normal
    derivative in y of Green's formula.  On the perturbed sphere the library
    picks the oracle's pivots (same ranks) and K x, K^T x equal the oracle's
    dense GCA matrix to 1e-10."""
    h = _lib()
    v, t = synth.perturbed_sphere(8, seed=3)
    K = oracle.dlp_dense(v, t, 4)
    A, info = gca.gca_dense_dlp(v, t, 16, m, eps, K)
    op = h.Operator(v, t, kernel="dlp", leaf=16, order_m=m, q_near=4, gca_tol=eps)
    st = op.info()
    assert st["row_coeffs"] == sum(info["row_ranks"].values())
    assert st["col_coeffs"] == sum(info["col_ranks"].values())
    x = synth.random_vector(len(v), 75)
    assert _rel(_product(op, x), A @ x) <= 1e-10
    xt = synth.random_vector(len(t), 76)
    torch = _torch()
    Y = torch.zeros(len(v), dtype=torch.float64, device="cuda")
    op.matvec(torch.tensor(xt, device="cuda"), Y, trans=True)
    torch.cuda.synchronize()
    assert _rel(Y.cpu().numpy(), A.T @ xt) <= 1e-10


def test_gca_error_falls_with_the_tolerance():
    """On the octahedral sphere (2,048 triangles, leaf 32) the error of the
    GCA product against the dense Galerkin matrix falls with the tolerance and
    the face quadrature order, and stays within a factor 3 of the oracle's
    GCA error for the same parameters (pivots may differ where the mesh's
    symmetries make entries tie)."""
    h = _lib()
    v, t = synth.octa_sphere(16)
    G = oracle.slp_dense(v, t, 4)
    x = synth.random_vector(len(t), 81)
    ref = G @ x
    errs = []
    for m, eps in ((2, 1e-2), (3, 1e-4), (4, 1e-6)):
        op = h.Operator(v, t, kernel="slp", leaf=32, order_m=m, q_near=4, gca_tol=eps)
        e = _rel(_product(op, x), ref)
        A, _ = gca.gca_dense(v, t, 32, m, eps, G)
        eo = _rel(A @ x, ref)
        print("GCA m=%d eps=%g: error %.3e (oracle %.3e), mean rank %.1f" % (m, eps, e, eo, op.info()["mean_rank_row"]))
        assert e <= 3 * eo + 1e-13, (m, eps, e, eo)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2], errs


def test_gca_mixed_precision_and_arguments():
    """The cross-approximation bases are not orthonormal, so an FP32 or BF16
    far field on them is refused (H2B_ENOTSUP), and so is their
    recompression into FP32 storage (FP64 only)."""
    h = _lib()
    v, t = synth.octa_sphere(16)
    for kernel in ("slp", "dlp"):
        for dt in ("f32", "bf16"):
            with pytest.raises(h.H2BError) as e:
                h.Operator(v, t, kernel=kernel, leaf=32, order_m=4, q_near=4, gca_tol=1e-6, farfield_dtype=dt)
            assert e.value.code == h.H2B_ENOTSUP
    with pytest.raises(h.H2BError) as e:
        h.Operator(v, t, kernel="slp", leaf=32, order_m=3, q_near=4, gca_tol=1e-4, recompress_tol=1e-6,
                   farfield_dtype="f32")
    assert e.value.code == h.H2B_ENOTSUP


def test_gca_operator_refuses_shape_derivatives():
    """The shape derivative differentiates the tensor Lagrange polynomials of
    the interpolation bases; cross-approximation bases are pivot-based, so
    both the geometry update and the gradient refuse them (H2B_ENOTSUP)."""
    import torch
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=2, q_near=4, gca_tol=1e-4)
    x = torch.ones(len(t), dtype=torch.float64, device="cuda")
    with pytest.raises(h.H2BError) as e:
        op.shape_grad(x, x)
    assert e.value.code == h.H2B_ENOTSUP
    with pytest.raises(h.H2BError) as e:
        op.set_geometry(v)
    assert e.value.code == h.H2B_ENOTSUP
