"""GPU parity: the HIP H^2 products against the CPU oracle, element by element.

* Far field disabled (every entry from the near-field quadrature): the GPU
  product equals the oracle's dense Galerkin matrix times x to rounding
  (bound 1e-10 relative to max|y|).
* Far field enabled: the GPU product equals the oracle's dense H^2 matrix
  (same trees, same interpolation, written out without transfer matrices) to
  rounding, and differs from the dense Galerkin matrix by the interpolation
  error of the order m.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import h2

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _lib():
    import paper_2001_05523_amd as h
    return h


def _run(op, x, trans=False, alpha=1.0, y0=None):
    torch = _torch()
    nout = op.shape[1] if trans else op.shape[0]
    X = torch.tensor(x, dtype=torch.float64, device="cuda")
    Y = (torch.zeros(nout, dtype=torch.float64, device="cuda") if y0 is None
         else torch.tensor(y0, dtype=torch.float64, device="cuda"))
    op.matvec(X, Y, alpha=alpha, trans=trans)
    torch.cuda.synchronize()
    return Y.cpu().numpy()


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


_dense_cache = {}


def _dense(s, kernel, q):
    key = (s, kernel, q)
    if key not in _dense_cache:
        v, t = synth.octa_sphere(s)
        _dense_cache[key] = (oracle.slp_dense if kernel == "slp" else oracle.dlp_dense)(v, t, q)
    return _dense_cache[key]


@pytest.mark.parametrize("s,leaf", [(2, 8), (4, 8), (8, 32), (8, 13)])
@pytest.mark.parametrize("kernel", ["slp", "dlp"])
@pytest.mark.parametrize("trans,copy", [(False, True), (True, True), (True, False)])
def test_dense_parity_far_disabled(s, leaf, kernel, trans, copy):
    """H^2 disabled: every entry is a near-field quadrature value, so the GPU
    product must equal the oracle's dense matrix to rounding (<= 1e-10).  The
    transposed product is checked from the transposed copy and from the
    column-wise read of the one copy."""
    h = _lib()
    v, t = synth.octa_sphere(s)
    q = 4
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, q_near=q, far_disabled=True, transposed_copy=copy)
    A = _dense(s, kernel, q)
    nin = A.shape[0] if trans else A.shape[1]
    x = synth.random_vector(nin, 101)
    y0 = synth.random_vector(A.shape[1] if trans else A.shape[0], 7)
    y = _run(op, x, trans=trans, alpha=-0.7, y0=y0)
    ref = y0 - 0.7 * ((A.T if trans else A) @ x)
    assert _maxrel(y, ref) <= 1e-10


def test_dense_parity_q6():
    h = _lib()
    v, t = synth.octa_sphere(4)
    op = h.Operator(v, t, kernel="dlp", leaf=16, q_near=6, far_disabled=True)
    K = oracle.dlp_dense(v, t, 6)
    x = synth.random_vector(len(v), 3)
    assert _maxrel(_run(op, x), K @ x) <= 1e-10


@pytest.mark.parametrize("kernel,s,leaf,m", [("slp", 8, 32, 3), ("slp", 8, 16, 2), ("slp", 16, 32, 4),
                                             ("dlp", 16, 16, 3), ("dlp", 16, 32, 4)])
def test_h2_parity_against_oracle_h2(kernel, s, leaf, m):
    """Interpolation far field: equal to the oracle's dense H^2 matrix to
    rounding; the error against the dense Galerkin matrix is the interpolation
    error of order m."""
    h = _lib()
    v, t = synth.octa_sphere(s)
    q = 4
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=q)
    assert op.blocks.nfar > 0
    A = _dense(s, kernel, q)
    H, _ = h2.h2_dense(v, t, kernel, leaf, m, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        x = synth.random_vector(nin, 101 + trans)
        y = _run(op, x, trans=trans)
        Hx = (H.T if trans else H) @ x
        Ax = (A.T if trans else A) @ x
        assert _maxrel(y, Hx) <= 1e-11
        err = np.linalg.norm(y - Ax) / np.linalg.norm(Ax)
        err_oracle = np.linalg.norm(Hx - Ax) / np.linalg.norm(Ax)
        print("%s m=%d trans=%d interpolation error %.3e (oracle H2 %.3e)"
              % (kernel, m, trans, err, err_oracle))
        assert abs(err - err_oracle) <= 1e-3 * err_oracle + 1e-12
        assert err_oracle < 1e-2


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_degenerate_meshes_against_dense_oracle(kernel):
    """Degenerate inputs against the oracle's H^2 matrix (the dense matrix
    when there is no far field) to rounding: one pair of triangles in each
    relation (one cluster), the octahedron with a leaf larger than the mesh,
    and a leaf of one triangle (deepest tree, far field down to single
    triangles).  Nothing may fail on them."""
    h = _lib()
    cases = [synth.single_pair(k) for k in ("edge", "vertex", "disjoint")]
    cases += [synth.octa_sphere(1), synth.octa_sphere(2)]
    for i, (v, t) in enumerate(cases):
        A = (oracle.slp_dense if kernel == "slp" else oracle.dlp_dense)(v, t, 4)
        for leaf in ((100,) if i < 4 else (1, 100)):
            op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=2, q_near=4)
            H, _ = h2.h2_dense(v, t, kernel, leaf, 2, near_matrix=A)
            if leaf == 100:
                assert op.info()["nfar"] == 0 and np.array_equal(H, A)
            for trans in (False, True):
                x = synth.random_vector(A.shape[0] if trans else A.shape[1], 341 + i)
                y = _run(op, x, trans=trans)
                ref = (H.T if trans else H) @ x
                scale = max(np.max(np.abs(ref)), 1e-300)
                assert np.max(np.abs(y - ref)) <= 1e-10 * scale + 1e-14, (i, leaf, trans)


def test_double_layer_vanishes_on_flat_plate():
    """On a plane <x - y, n_y> = 0, so every entry of K vanishes (the oracle's
    dense K is exactly zero) and so must the nearfield product, to rounding.
    The far field is the normal derivative of the interpolant; across a flat
    cluster the Chebyshev points in the normal direction collapse onto a
    widened degenerate box side, so it is only small (interpolation error
    amplified by that degenerate width), not zero."""
    h = _lib()
    v, t = synth.flat_plate(8)
    g = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4, far_disabled=True)
    near = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4, far_disabled=True)
    full = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
    assert full.info()["nfar"] > 0
    assert np.max(np.abs(oracle.dlp_dense(v, t, 4))) == 0.0
    x = synth.random_vector(near.shape[1], 351)
    yg = _run(g, synth.random_vector(g.shape[1], 352))
    assert np.max(np.abs(_run(near, x))) <= 1e-12 * np.max(np.abs(yg))
    assert np.max(np.abs(_run(full, x))) <= 1e-3 * np.max(np.abs(yg))


def test_largest_order_and_quadrature():
    """Order 6 (k = 216 coefficients per cluster, panels wider than a wave)
    and q_near 16, the largest the library accepts, against the oracle's H^2."""
    h = _lib()
    v, t = synth.octa_sphere(4)
    A = oracle.slp_dense(v, t, 16)
    op = h.Operator(v, t, kernel="slp", leaf=8, order_m=6, q_near=16)
    assert op.info()["nfar"] > 0 and op.info()["max_rank_row"] == 216
    H, _ = h2.h2_dense(v, t, "slp", 8, 6, near_matrix=A)
    for trans in (False, True):
        x = synth.random_vector(A.shape[0], 361 + trans)
        assert _maxrel(_run(op, x, trans=trans), (H.T if trans else H) @ x) <= 1e-11


def test_leaves_larger_than_64_keep_the_full_nearfield():
    """The once-per-pair nearfield needs leaves of at most 64; with larger
    leaves G is assembled without it and stays exact."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=200, order_m=2, q_near=4)
    assert op.info()["near_sym_entries"] == 0
    A = _dense(8, "slp", 4)
    H, _ = h2.h2_dense(v, t, "slp", 200, 2, near_matrix=A)
    x = synth.random_vector(A.shape[1], 371)
    assert _maxrel(_run(op, x), H @ x) <= 1e-11


@pytest.mark.parametrize("kernel,s,leaf", [("slp", 16, 16), ("dlp", 16, 16), ("slp", 16, 32)])
def test_recompressed_against_oracle_h2(kernel, s, leaf):
    """Algebraic recompression of the order-4 interpolation bases to 1e-6
    (relative per cluster): the product stays within a small multiple of the
    tolerance of the oracle's (uncompressed) H^2 matrix while the ranks drop."""
    h = _lib()
    v, t = synth.octa_sphere(s)
    q, m, tol = 4, 4, 1e-6
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=q, recompress_tol=tol)
    info = op.info()
    assert info["mean_rank_row"] < m ** 3 and info["max_rank_row"] <= m ** 3
    A = _dense(s, kernel, q)
    H, _ = h2.h2_dense(v, t, kernel, leaf, m, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        x = synth.random_vector(nin, 5 + trans)
        y = _run(op, x, trans=trans)
        Hx = (H.T if trans else H) @ x
        err = np.linalg.norm(y - Hx) / np.linalg.norm(Hx)
        print("%s trans=%d recompressed vs oracle H2: %.3e, mean rank %.1f / %.1f"
              % (kernel, trans, err, info["mean_rank_row"], info["mean_rank_col"]))
        assert err <= 20 * tol


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_recompressed_order5_against_oracle_h2(kernel):
    """Recompression of order-5 interpolation bases (k = 125 > 64: the tiled
    sandwich and Gram kernels and the orthogonalisation from the stored
    transfer matrices): within a small multiple of the tolerance of the
    oracle's (uncompressed) H^2 matrix, with lower ranks."""
    h = _lib()
    s, q, m, tol, leaf = 16, 4, 5, 1e-6, 16
    v, t = synth.octa_sphere(s)
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=q, recompress_tol=tol)
    info = op.info()
    assert info["max_rank_row"] < m ** 3 and info["mean_rank_row"] < 64
    A = _dense(s, kernel, q)
    H, _ = h2.h2_dense(v, t, kernel, leaf, m, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        x = synth.random_vector(nin, 25 + trans)
        y = _run(op, x, trans=trans)
        Hx = (H.T if trans else H) @ x
        err = np.linalg.norm(y - Hx) / np.linalg.norm(Hx)
        print("%s trans=%d order-5 recompressed vs oracle H2: %.3e, mean rank %.1f, max %d"
              % (kernel, trans, err, info["mean_rank_row"], info["max_rank_row"]))
        assert err <= 20 * tol


def test_recompressed_mixed_precision():
    """FP32 storage of the recompressed (orthonormal) bases and couplings stays
    within 1e-5 of the FP64 recompressed product."""
    h = _lib()
    v, t = synth.octa_sphere(32)
    for kernel in ("slp", "dlp"):
        op64 = h.Operator(v, t, kernel=kernel, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6)
        op32 = h.Operator(v, t, kernel=kernel, leaf=32, order_m=4, q_near=4, recompress_tol=1e-6,
                          farfield_dtype="f32")
        for trans in (False, True):
            nin = op64.shape[0] if trans else op64.shape[1]
            x = synth.random_vector(nin, 13)
            y64 = _run(op64, x, trans=trans)
            y32 = _run(op32, x, trans=trans)
            d = np.linalg.norm(y32 - y64) / np.linalg.norm(y64)
            print("%s trans=%d mixed vs fp64 (recompressed): %.3e" % (kernel, trans, d))
            assert d <= 1e-5


def test_reduced_precision_needs_orthonormal_bases():
    """FP32 and BF16 far fields are refused (H2B_ENOTSUP) where the bases are
    not orthonormal: plain interpolation (recompress_tol = 0) and the Green
    cross approximation.  Their rounding would be amplified by the basis
    condition beyond the 1e-5 of the precision form."""
    h = _lib()
    v, t = synth.octa_sphere(4)
    for kernel in ("slp", "dlp"):
        for dt in ("f32", "bf16"):
            for kw in (dict(), dict(gca_tol=1e-4)):
                with pytest.raises(h.H2BError) as e:
                    h.Operator(v, t, kernel=kernel, leaf=8, order_m=3, q_near=4, farfield_dtype=dt, **kw)
                assert e.value.code == h.H2B_ENOTSUP, (kernel, dt, kw)
            h.Operator(v, t, kernel=kernel, leaf=8, order_m=3, q_near=4, farfield_dtype=dt, recompress_tol=1e-6)


def test_multiple_right_hand_sides():
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
    nr, nc = op.shape
    X = torch.tensor(synth.random_vector(nc + 5, 5, cols=3), device="cuda")[:nc]
    Y = torch.zeros((nr + 3, 3), dtype=torch.float64, device="cuda").t().contiguous().t()[:nr]
    op.matvec(X, Y, alpha=2.0)
    torch.cuda.synchronize()
    for c in range(3):
        y1 = _run(op, X[:, c].cpu().numpy(), alpha=2.0)
        np.testing.assert_allclose(Y[:, c].cpu().numpy(), y1, rtol=0, atol=1e-13 * np.abs(y1).max())


def test_argument_errors_leave_y_untouched():
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(4)
    op = h.Operator(v, t, kernel="slp", leaf=8, order_m=2)
    x = torch.ones(len(t), dtype=torch.float64, device="cuda")
    y = torch.full((len(t),), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(h.H2BError):
        h._check(h.h2b_matvec(op.handle, 0, 1.0, h._vp(x.data_ptr()), len(t) - 1,
                              h._vp(y.data_ptr()), len(t), 1, None))
    with pytest.raises(h.H2BError):
        h._check(h.h2b_matvec(op.handle, 0, 1.0, h._vp(x.data_ptr()), len(t),
                              h._vp(x.data_ptr()), len(t), 1, None))
    torch.cuda.synchronize()
    assert torch.all(y == 3.0)
    with pytest.raises(h.H2BError):
        h.Operator(v, t, kernel="slp", leaf=8, order_m=9)
    with pytest.raises(h.H2BError):
        h.Operator(v, t, kernel="slp", leaf=8, q_near=1)


def test_single_hip_runtime_loaded():
    """The library and torch share one HIP runtime in the process."""
    torch = _torch()
    _lib()
    torch.zeros(1, device="cuda")
    maps = open("/proc/self/maps").read().splitlines()
    libs = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    assert len(libs) == 1, libs
    assert any("libh2bem.so" in ln for ln in maps)


def _run_block(op, X, trans=False, alpha=1.0):
    """X: (n, nrhs) numpy array; returns op(A) X through one block product."""
    torch = _torch()
    nout = op.shape[1] if trans else op.shape[0]
    Xd = torch.tensor(np.asfortranarray(X), device="cuda").t().contiguous().t()
    Yd = torch.zeros((X.shape[1], nout), dtype=torch.float64, device="cuda").t()
    op.matvec(Xd, Yd, alpha=alpha, trans=trans)
    torch.cuda.synchronize()
    return Yd.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [64, 37])
def test_many_right_hand_sides(dtype, nrhs):
    """Blocks of right-hand sides (GEMM form, matrix cores for the FP32/BF16
    coupling) agree with the single-vector FP64 products of the same
    (recompressed, orthonormal-basis) operator: FP64 to rounding, FP32 to
    1e-5, BF16 within its 8-bit mantissa."""
    h = _lib()
    v, t = synth.octa_sphere(16)
    for kernel in ("slp", "dlp"):
        kw = dict(kernel=kernel, leaf=16, order_m=4, q_near=4, recompress_tol=1e-6)
        op = h.Operator(v, t, farfield_dtype=dtype, **kw)
        ref_op = op if dtype == "f64" else h.Operator(v, t, **kw)
        for trans in (False, True):
            nin = op.shape[0] if trans else op.shape[1]
            X = synth.random_vector(nin, 301, cols=nrhs)
            Y = _run_block(op, X, trans=trans, alpha=0.5)
            for c in (0, nrhs // 2, nrhs - 1):
                y1 = _run(ref_op, X[:, c], trans=trans, alpha=0.5)
                d = np.linalg.norm(Y[:, c] - y1) / np.linalg.norm(y1)
                bound = {"f64": 1e-12, "f32": 1e-5, "bf16": 5e-3}[dtype]
                assert d <= bound, (kernel, trans, c, d)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_transposed_copy_matches_column_read(dtype):
    """A^T x from the transposed copies (row kernels) and from the column-wise
    read of the single copy use the same stored values, so they agree to
    rounding, for one vector and for a block of 16.  The BF16 block product
    from the copy runs on matrix cores, which also round the cluster
    coefficients to BF16: that bound is BF16's."""
    h = _lib()
    v, t = synth.octa_sphere(16)
    bound = {"f64": 1e-13, "f32": 1e-6, "bf16": 1e-6}[dtype]
    block_bound = {"f64": 1e-13, "f32": 1e-6, "bf16": 5e-3}[dtype]
    for kernel in ("slp", "dlp"):
        kw = dict(kernel=kernel, leaf=16, order_m=4, q_near=4, recompress_tol=1e-6, farfield_dtype=dtype)
        a = h.Operator(v, t, transposed_copy=True, **kw)
        b = h.Operator(v, t, transposed_copy=False, **kw)
        assert a.info()["bytes_transposed"] > 0 and b.info()["bytes_transposed"] == 0
        x = synth.random_vector(a.shape[0], 311)
        ya, yb = _run(a, x, trans=True), _run(b, x, trans=True)
        d = np.linalg.norm(ya - yb) / np.linalg.norm(yb)
        assert d <= bound, (kernel, d)
        X = synth.random_vector(a.shape[0], 312, cols=16)
        Ya, Yb = _run_block(a, X, trans=True), _run_block(b, X, trans=True)
        d = np.linalg.norm(Ya - Yb) / np.linalg.norm(Yb)
        assert d <= block_bound, (kernel, "block", d)


@pytest.mark.parametrize("far_disabled,tol", [(True, 0.0), (False, 1e-6)])
def test_once_per_pair_nearfield_matches_full(far_disabled, tol):
    """G x and G^T x from the nearfield stored once per pair of leaves (plus
    the corrections of the touching pairs across leaves) equal the products
    from the full nearfield to rounding; sizes span several leaves and a
    ragged last leaf (leaf 13)."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    kw = dict(kernel="slp", leaf=13, order_m=3, q_near=4, far_disabled=far_disabled, recompress_tol=tol)
    a = h.Operator(v, t, symmetric_near=True, **kw)
    b = h.Operator(v, t, symmetric_near=False, **kw)
    ia, ib = a.info(), b.info()
    assert ia["near_sym_entries"] > 0 and ib["near_sym_entries"] == 0
    assert ia["near_sym_entries"] < 0.75 * ia["near_entries"]
    assert ia["near_sym_corrections"] > 0
    for trans in (False, True):
        x = synth.random_vector(a.shape[0], 331 + trans)
        ya, yb = _run(a, x, trans=trans), _run(b, x, trans=trans)
        assert _maxrel(ya, yb) <= 1e-13, (trans, _maxrel(ya, yb))


@pytest.mark.parametrize("order,tol,dtype", [(3, 0.0, "f64"), (4, 0.0, "f64"), (4, 1e-6, "f64"),
                                             (4, 1e-6, "f32"), (5, 0.0, "f64")])
def test_once_per_pair_coupling_matches_full(order, tol, dtype):
    """G x and G^T x with the far field stored once per pair of clusters
    (S_ts for s > t, S_st taken as its transpose) equal the products from the
    full coupling panels to rounding (FP64), or to FP32 summation-order error
    for an FP32 far field.  The stored pairs hold exactly half the coupling
    entries (blocks (t, s) and (s, t) have the same shape); with order 4
    (rank 64) the panels are wider than one 256-column pass, and order 5
    (rank 125) has more rows than a wave has lanes."""
    h = _lib()
    v, t = synth.octa_sphere(16)
    kw = dict(kernel="slp", leaf=16, order_m=order, q_near=4, recompress_tol=tol, farfield_dtype=dtype)
    a = h.Operator(v, t, symmetric_near=True, **kw)
    b = h.Operator(v, t, symmetric_near=False, **kw)
    ia, ib = a.info(), b.info()
    assert ib["cpl_sym_entries"] == 0 and ia["cpl_sym_entries"] > 0
    assert 2 * ia["cpl_sym_entries"] == ia["coupling_entries"]
    assert ia["cpl_sym_columns"] > 0
    for trans in (False, True):
        x = synth.random_vector(a.shape[0], 341 + trans)
        ya, yb = _run(a, x, trans=trans), _run(b, x, trans=trans)
        bound = 1e-13 if dtype == "f64" else 1e-6
        assert _maxrel(ya, yb) <= bound, (trans, _maxrel(ya, yb))


def test_once_per_pair_coupling_only_where_it_applies():
    """BF16 couplings (on recompressed bases) and evaluated couplings keep
    the full coupling panels or none; the double-layer operator has no such
    storage."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    for kw in (dict(kernel="slp", order_m=3, farfield_dtype="bf16", recompress_tol=1e-6),
               dict(kernel="slp", order_m=3, recompute_coupling=True), dict(kernel="dlp", order_m=3)):
        op = h.Operator(v, t, leaf=16, q_near=4, **kw)
        assert op.info()["cpl_sym_entries"] == 0, kw


def test_phase_timing_brackets_the_product():
    """Per-phase event timing with the nearfield on its own stream: every phase
    lies inside the whole product, and timing does not change the result."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="dlp", leaf=16, order_m=3, q_near=4)
    for trans in (False, True):
        x = synth.random_vector(op.shape[0] if trans else op.shape[1], 321)
        y0 = _run(op, x, trans=trans)
        op.set_timing(True)
        ys = [_run(op, x, trans=trans) for _ in range(3)]
        ph = op.phase_times()
        op.set_timing(False)
        for y in ys:
            assert np.array_equal(y, y0)
        assert set(ph) == {"gather", "forward", "coupling", "backward", "nearfield", "scatter", "total"}
        assert all(v > 0 for v in ph.values()), ph
        far = ph["gather"] + ph["forward"] + ph["coupling"] + ph["backward"]
        assert ph["total"] >= max(far, ph["nearfield"]) * (1 - 1e-6), ph
        # every phase on the caller's stream: same result, phases in sequence
        op.set_overlap(False)
        op.set_timing(True)
        y1 = _run(op, x, trans=trans)
        ph = op.phase_times()
        op.set_timing(False)
        op.set_overlap(True)
        assert np.array_equal(y1, y0)
        far = ph["gather"] + ph["forward"] + ph["coupling"] + ph["backward"]
        assert ph["total"] >= far + ph["nearfield"] + ph["scatter"] - 1e-3, ph


def test_tuner_picks_a_tile_and_products_stay_exact():
    h = _lib()
    v, t = synth.octa_sphere(16)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=4, q_near=4, farfield_dtype="f32",
                    recompress_tol=1e-6)
    us = op.tune(64)
    assert us > 0
    X = synth.random_vector(op.shape[1], 303, cols=64)
    Y = _run_block(op, X)
    for c in (0, 63):
        y1 = _run(op, X[:, c])
        assert np.linalg.norm(Y[:, c] - y1) / np.linalg.norm(y1) <= 1e-5


def test_batched_graph_of_uneven_meshes():
    """Sixteen meshes of uneven size (spheres of random radius and ellipsoids
    with random semi-axes, 2 s^2 ... triangles) captured into one graph: every
    replay is bitwise the first one, with eager work and synchronisations
    between replays, and equals the eager products up to FP32 rounding.  The
    far field is FP32 and the merged launches sum the transformations in
    another order than the per-level launches of one product: a few FP32 ulps
    (2^-24 = 6e-8) of the largest entry, bounded here by 1e-6 of it."""
    torch = _torch()
    h = _lib()
    rng = np.random.default_rng(302)
    ops, xs, ys, refs = [], [], [], []
    for k in range(16):
        s = int(rng.integers(4, 13))
        if k % 2 == 0:
            r = rng.uniform(0.5, 2.0)
            v, t = synth.ellipsoid(s, r, r, r)
        else:
            a, b, c = rng.uniform(0.5, 2.0, size=3)
            v, t = synth.ellipsoid(s, a, b, c)
        kern = "slp" if k % 3 else "dlp"
        op = h.Operator(v, t, kernel=kern, leaf=16, order_m=3, q_near=4, farfield_dtype="f32",
                        recompress_tol=1e-6)
        x = torch.tensor(synth.random_vector(op.shape[1], 303 + k), device="cuda")
        y = torch.zeros(op.shape[0], dtype=torch.float64, device="cuda")
        ref = torch.zeros_like(y)
        op.matvec(x, ref)
        ops.append(op)
        xs.append(x)
        ys.append(y)
        refs.append(ref)
    torch.cuda.synchronize()
    batch = h.Batch(list(zip(ops, xs, ys)))
    first = None
    for rep in range(4):
        for y in ys:
            y.zero_()
        torch.cuda.synchronize()
        batch.launch()
        torch.cuda.synchronize()
        got = [y.cpu().numpy() for y in ys]
        if first is None:
            first = got
        for g, f, ref in zip(got, first, refs):
            np.testing.assert_array_equal(g, f)
            np.testing.assert_allclose(g, ref.cpu().numpy(), rtol=0, atol=1e-6 * float(ref.abs().max()))
        # eager work in between replays
        ops[0].matvec(xs[0], refs[0], alpha=0.0)
        torch.cuda.synchronize()


def test_batch_rejects_repeated_operator():
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(4)
    op = h.Operator(v, t, kernel="slp", leaf=8, order_m=2)
    x = torch.ones(len(t), dtype=torch.float64, device="cuda")
    y1 = torch.zeros_like(x)
    y2 = torch.zeros_like(x)
    with pytest.raises(h.H2BError):
        h.Batch([(op, x, y1), (op, x, y2)])


@pytest.mark.parametrize("nrhs", [64, 37])
@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_block_product_against_oracle_h2(kernel, nrhs):
    """Blocks of right-hand sides in FP64 (block GEMMs, nearfield and coupling
    on matrix cores) against the oracle's dense H^2 matrix times the same
    block, element by element to rounding, for A X and A^T X; the mesh spans
    many leaves and the 37-column block leaves a ragged tail of the 64-wide
    block."""
    h = _lib()
    s, leaf, m = 16, 16, 4
    v, t = synth.octa_sphere(s)
    op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=m, q_near=4)
    A = _dense(s, kernel, 4)
    H, _ = h2.h2_dense(v, t, kernel, leaf, m, near_matrix=A)
    for trans in (False, True):
        nin = A.shape[0] if trans else A.shape[1]
        X = synth.random_vector(nin, 381 + trans, cols=nrhs)
        Y = _run_block(op, X, trans=trans, alpha=0.5)
        ref = 0.5 * ((H.T if trans else H) @ X)
        assert np.max(np.abs(Y - ref)) <= 1e-11 * np.max(np.abs(ref)), (trans, _maxrel(Y, ref))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_recompressed_block_product_against_oracle_h2(dtype):
    """Recompressed order-4 operators (orthonormal bases) with FP64, FP32 and
    BF16 far fields, 64 right-hand sides, against the oracle's dense
    (uncompressed) H^2 matrix: every column within the recompression bound
    (20 x 1e-6) plus the rounding of the storage type (FP32 1e-5, BF16 5e-3)."""
    h = _lib()
    s, leaf = 16, 16
    v, t = synth.octa_sphere(s)
    for kernel in ("slp", "dlp"):
        op = h.Operator(v, t, kernel=kernel, leaf=leaf, order_m=4, q_near=4, recompress_tol=1e-6,
                        farfield_dtype=dtype)
        A = _dense(s, kernel, 4)
        H, _ = h2.h2_dense(v, t, kernel, leaf, 4, near_matrix=A)
        bound = 20e-6 + {"f64": 0.0, "f32": 1e-5, "bf16": 5e-3}[dtype]
        for trans in (False, True):
            nin = A.shape[0] if trans else A.shape[1]
            X = synth.random_vector(nin, 391 + trans, cols=64)
            Y = _run_block(op, X, trans=trans)
            ref = (H.T if trans else H) @ X
            err = np.linalg.norm(Y - ref, axis=0) / np.linalg.norm(ref, axis=0)
            print("%s %s trans=%d: max column error %.3e" % (kernel, dtype, trans, err.max()))
            assert err.max() <= bound, (kernel, trans, err.max())


def test_batch_survives_tuning_after_creation():
    """A batch captures the block work vectors of its operators; tuning an
    operator afterwards (which selects another block width) and wider
    products must not move them, so the replays still equal eager
    products."""
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(8)
    ops = [h.Operator(v, t, kernel=k, leaf=16, order_m=3, q_near=4) for k in ("slp", "dlp")]
    items, refs = [], []
    for i, op in enumerate(ops):
        X = torch.tensor(synth.random_vector(op.shape[1], 395 + i, cols=16), device="cuda").t().contiguous().t()
        Y = torch.zeros((16, op.shape[0]), dtype=torch.float64, device="cuda").t()
        R = torch.zeros((16, op.shape[0]), dtype=torch.float64, device="cuda").t()
        op.matvec(X, R)
        items.append((op, X, Y))
        refs.append(R)
    batch = h.Batch(items)
    for op in ops:
        op.tune(64)
        Xw = torch.tensor(synth.random_vector(op.shape[1], 397, cols=64), device="cuda").t().contiguous().t()
        op.matvec(Xw, torch.zeros((64, op.shape[0]), dtype=torch.float64, device="cuda").t())
    torch.cuda.synchronize()
    for rep in range(2):
        for _, _, Y in items:
            Y.zero_()
        batch.launch()
        torch.cuda.synchronize()
        for (_, _, Y), R in zip(items, refs):
            np.testing.assert_allclose(Y.cpu().numpy(), R.cpu().numpy(), rtol=0,
                                       atol=1e-12 * float(R.abs().max()))
