"""The H-Cholesky preconditioner on the device: the substitutions of the
flattened program against the host solve of the same factor, the factor of
the H^2 operator converted on the host against the oracle's dense matrices,
and preconditioned CG on the device."""
import numpy as np
import pytest

import oracle
import synth
from oracle import h2 as oh2

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _lib():
    import paper_2001_05523_amd as h
    return h


def _dev(a):
    return _torch().tensor(np.ascontiguousarray(a), device="cuda")


def _apply(P, r):
    torch = _torch()
    z = torch.zeros(len(r), dtype=torch.float64, device="cuda")
    P.apply(_dev(r), z)
    torch.cuda.synchronize()
    return z.cpu().numpy()


def _lower_sym(A):
    return np.tril(A) + np.tril(A, -1).T


@pytest.mark.parametrize("s,leaf,eps", [(4, 8, 0.0), (8, 16, 0.0), (8, 16, 1e-3), (16, 16, 1e-2), (8, 5, 1e-4)])
def test_device_substitutions_equal_host_solve(s, leaf, eps):
    """Same factor, same arithmetic per entry, other summation order: the
    device and host solves agree to rounding."""
    h = _lib()
    v, t = synth.octa_sphere(s)
    G = oracle.slp_dense(v, t, 4)
    T = h.Tree(h.Mesh(v, t), 0, leaf)
    P = h.HChol.from_dense(h.Blocks(T, T, 1.0), G, eps)
    for seed in (21, 22):
        r = synth.random_vector(len(t), seed)
        zh = P.solve_host(r)
        zd = _apply(P, r)
        assert np.linalg.norm(zd - zh) <= 1e-12 * np.linalg.norm(zh), seed
    info = P.info()
    assert info["steps"] > 0 and info["tasks"] >= info["steps"]


def test_device_substitutions_of_a_larger_operator():
    """8,192 triangles: low-rank factors longer than one coefficient piece
    (1,024 rows), computed in pieces and summed; device equals host."""
    h = _lib()
    v, t = synth.octa_sphere(32)
    op = h.Operator(v, t, kernel="slp", leaf=32, order_m=4, q_near=4, recompress_tol=1e-6)
    P = h.HChol(op, 1e-3)
    r = synth.random_vector(len(t), 27)
    zh = P.solve_host(r)
    zd = _apply(P, r)
    assert np.linalg.norm(zd - zh) <= 1e-12 * np.linalg.norm(zh)


def test_operator_without_far_field_gives_the_cholesky_solve():
    """Far field disabled: the converted H-matrix is the lower triangle of
    the dense Galerkin G of the oracle (entries equal to 1e-10), so with
    eps = 0 the device solve is that matrix's solve."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=16, q_near=4, far_disabled=True)
    P = h.HChol(op, 0.0)
    G = oracle.slp_dense(v, t, 4)
    perm = h.Tree(h.Mesh(v, t), 0, 16).arrays()["perm"]
    Gl = _lower_sym(G[np.ix_(perm, perm)])
    r = synth.random_vector(len(t), 23)
    zref = np.empty_like(r)
    zref[perm] = np.linalg.solve(Gl, r[perm])
    z = _apply(P, r)
    assert np.linalg.norm(z - zref) <= 1e-8 * np.linalg.norm(zref)


@pytest.mark.parametrize("tol", [0.0, 1e-6])
def test_operator_factor_against_oracle_h2(tol):
    """With the far field: the farfield blocks V_t S_ts V_s^T become low-rank
    blocks through the explicit parent bases; with eps = 0 the factor solves
    the oracle's dense H^2 matrix (lower triangle), for plain interpolation
    and for recompressed bases (then to the recompression tolerance)."""
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4, recompress_tol=tol)
    P = h.HChol(op, 0.0)
    A, _ = oh2.h2_dense(v, t, "slp", 16, 3, near_matrix=oracle.slp_dense(v, t, 4))
    perm = h.Tree(h.Mesh(v, t), 0, 16).arrays()["perm"]
    Al = _lower_sym(A[np.ix_(perm, perm)])
    r = synth.random_vector(len(t), 24)
    zref = np.empty_like(r)
    zref[perm] = np.linalg.solve(Al, r[perm])
    z = _apply(P, r)
    bound = 1e-8 if tol == 0.0 else 1e-3
    err = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    print("recompress_tol %.0e: %.2e" % (tol, err))
    assert err <= bound


def test_factor_of_gca_operator_inverts_the_product():
    """The Green cross approximation keeps its bases in the same panels
    (V_t^T per leaf, [E_1^T | E_2^T] per parent), so its operator converts
    the same way: with eps = 0, G z for z = (L L^T)^{-1} r gives back r up to
    the asymmetry of the quadrature of touching pairs (about 1e-7 relative,
    times the condition number of G here, about 100)."""
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(8)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=3, q_near=4, gca_tol=1e-6, symmetric_near=False)
    P = h.HChol(op, 0.0)
    r = _dev(synth.random_vector(len(t), 26))
    z = torch.zeros_like(r)
    P.apply(r, z)
    back = torch.zeros_like(r)
    op.matvec(z, back)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(back - r) / torch.linalg.norm(r))
    print("GCA: |G z - r| / |r| = %.2e" % err)
    assert err <= 1e-4


def test_preconditioned_cg_on_the_device():
    """PCG with the factor: few iterations, the same solution as plain CG,
    and the same bits with and without graph replay (G with the plain
    nearfield storage, whose reductions have a fixed order; the
    substitutions run in one workgroup in a fixed order)."""
    torch = _torch()
    h = _lib()
    v, t = synth.octa_sphere(16)
    op = h.Operator(v, t, kernel="slp", leaf=16, order_m=4, q_near=4, symmetric_near=False)
    P = h.HChol(op, 1e-2)
    b = _dev(synth.random_vector(len(t), 25))
    x0 = torch.zeros_like(b)
    r0 = op.cg(b, x0, tol=1e-10, max_iter=1000)
    sols = []
    for graph in (True, False):
        x = torch.zeros_like(b)
        r = op.cg(b, x, tol=1e-10, max_iter=1000, precond="hchol", hchol=P, use_graph=graph)
        assert r["status"] == "converged"
        sols.append(x.cpu().numpy())
        print("cg %d iterations, pcg %d (graph %s)" % (r0["iterations"], r["iterations"], graph))
        assert r["iterations"] <= 15 and 4 * r["iterations"] < r0["iterations"]
    ref = x0.cpu().numpy()
    for xs in sols:
        assert np.linalg.norm(xs - ref) <= 1e-7 * np.linalg.norm(ref)
    assert np.array_equal(sols[0], sols[1])


def test_rejected_configurations():
    h = _lib()
    v, t = synth.octa_sphere(4)
    for kw in (dict(kernel="dlp"), dict(kernel="slp", farfield_dtype="f32", recompress_tol=1e-6),
               dict(kernel="slp", recompute_coupling=True)):
        op = h.Operator(v, t, leaf=8, order_m=2, q_near=4, **kw)
        with pytest.raises(h.H2BError):
            h.HChol(op, 1e-3)
    op = h.Operator(v, t, kernel="slp", leaf=8, order_m=2, q_near=4)
    with pytest.raises(h.H2BError):
        h.HChol(op, float("nan"))
