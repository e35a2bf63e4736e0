"""Pins of the oracle's Green cross approximation (Section 4) against facts
that do not come from the oracle itself: Green's representation formula on
the auxiliary box reproduces the kernel, the cross approximation reproduces a
matrix of exact low rank, the bases interpolate on their pivot rows, and the
GCA matrix converges to the dense Galerkin matrix as the tolerance falls."""
import math

import numpy as np
import pytest

import oracle
import oracle.h2
import synth
from oracle import gca


def _green_quadrature_error(m):
    """Max relative error of the discretised Green formula for x in the unit
    box and y in a box several diameters away."""
    lo, hi = gca.omega_box(np.zeros(3), np.ones(3))
    Z, W, N = gca.face_rule(lo, hi, m)
    rng = np.random.default_rng(0)
    err = 0.0
    for _ in range(20):
        x = rng.uniform(0.0, 1.0, 3)
        y = np.array([6.0, 0.5, -2.0]) + rng.uniform(0.0, 1.0, 3)
        dxz = x - Z
        rxz = np.linalg.norm(dxz, axis=1)
        dzy = Z - y
        rzy = np.linalg.norm(dzy, axis=1)
        g_xz = 1.0 / (4 * math.pi * rxz)
        dn_xz = np.einsum("kd,kd->k", dxz, N) / (4 * math.pi * rxz ** 3)   # n_z . grad_z g(x, z)
        g_zy = 1.0 / (4 * math.pi * rzy)
        dn_zy = -np.einsum("kd,kd->k", dzy, N) / (4 * math.pi * rzy ** 3)  # n_z . grad_z g(z, y)
        approx = np.sum(W * g_xz * dn_zy) - np.sum(W * dn_xz * g_zy)
        exact = 1.0 / (4 * math.pi * np.linalg.norm(x - y))
        err = max(err, abs(approx - exact) / exact)
    return err


def test_face_rule_integrates_the_box_surface():
    """Six faces of m x m Gauss points: the weights add up to the surface
    area, and the normals are outward (the flux of x through the boundary is
    three times the volume, divergence theorem)."""
    lo, hi = np.array([-1.0, 0.0, 2.0]), np.array([0.5, 2.0, 2.5])
    Z, W, N = gca.face_rule(lo, hi, 3)
    e = hi - lo
    assert W.sum() == pytest.approx(2 * (e[0] * e[1] + e[1] * e[2] + e[0] * e[2]), rel=1e-14)
    assert np.sum(W * np.einsum("kd,kd->k", Z, N)) == pytest.approx(3 * np.prod(e), rel=1e-13)


def test_green_formula_on_the_box_converges():
    """Green's representation formula (Section 1) applied on omega_t with the
    face rule reproduces g(x, y) for x inside and y outside, the error
    falling with the quadrature order (Section 4)."""
    errs = [_green_quadrature_error(m) for m in (2, 4, 6, 8, 10)]
    assert all(errs[i] > 3 * errs[i + 1] for i in range(4)), errs
    assert errs[-1] < 1e-5, errs


def test_cross_approximation_reproduces_low_rank_matrices():
    """A rank-5 matrix is reproduced after five steps by the skeleton
    L|_{. x sigma} (L|_{tau x sigma})^{-1} L|_{tau x .}."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 5)) @ rng.standard_normal((5, 40))
    tau, sigma = gca.aca_full(A, 1e-12)
    assert len(tau) == 5
    S = A[:, sigma] @ np.linalg.solve(A[np.ix_(tau, sigma)], A[tau, :])
    assert np.max(np.abs(S - A)) <= 1e-12 * np.max(np.abs(A))


def test_bases_interpolate_on_their_pivots():
    """V_t restricted to the pivot rows is the identity (algebraic
    interpolation, Section 4), for leaves and for the stacked transfers, up
    to the rounding of the solve with the pivot block (whose condition grows
    as the tolerance falls: 5e-12 at 1e-4, 5e-10 at 1e-6)."""
    v, t = synth.perturbed_sphere(4, seed=2)
    cent = v[t].mean(axis=1)
    root, perm, clusters = oracle.h2.cluster_tree(cent, 8)
    oracle.h2.support_boxes(clusters, v, t, "P0")
    hat, V = gca.gca_bases(v, t, clusters, perm, 3, 1e-4)
    for c in clusters:
        rows = np.concatenate([hat[ch.id] for ch in c.children]) if c.children else perm[c.begin:c.end]
        pos = [int(np.where(rows == i)[0][0]) for i in hat[c.id]]
        assert np.max(np.abs(V[c.id][pos] - np.eye(len(pos)))) <= 1e-10


def test_gca_converges_to_the_galerkin_matrix():
    """The GCA matrix approaches the dense Galerkin G as the tolerance and
    the face order grow (errors of G x, 512 triangles, leaf 16)."""
    v, t = synth.octa_sphere(8)
    G = oracle.slp_dense(v, t, 4)
    x = synth.random_vector(len(t), 1)
    errs = []
    for m, eps in ((2, 1e-2), (3, 1e-4), (4, 1e-6)):
        A, info = gca.gca_dense(v, t, 16, m, eps, G)
        assert info["far"] > 0
        errs.append(np.linalg.norm(A @ x - G @ x) / np.linalg.norm(G @ x))
    assert errs[0] > 100 * errs[1] and errs[1] > 100 * errs[2], errs
    assert errs[0] < 1e-2, errs


def test_gca_double_layer_converges_to_the_galerkin_matrix():
    """K with vertex-cluster bases from the normal derivative in y of Green's
    formula: the GCA matrix approaches the dense Galerkin K as the tolerance
    and the face order grow (a wrong sign or term in the second derivative
    would stop the convergence)."""
    v, t = synth.octa_sphere(8)
    K = oracle.dlp_dense(v, t, 4)
    x = synth.random_vector(len(v), 2)
    errs = []
    for m, eps in ((2, 1e-2), (3, 1e-4)):
        A, info = gca.gca_dense_dlp(v, t, 16, m, eps, K)
        assert info["far"] > 0
        errs.append(np.linalg.norm(A @ x - K @ x) / np.linalg.norm(K @ x))
    assert errs[0] > 50 * errs[1], errs
    assert errs[1] < 1e-5, errs


def test_gca_single_layer_symmetric_off_touching_pairs():
    """The cross approximation of G takes its couplings from G's entries
    between pivot triangles of admissible clusters (never touching) and uses
    one nested basis for rows and columns, so the GCA matrix is symmetric to
    rounding off the touching pairs, as G is; G's once-per-pair storage of
    the GCA far field relies on this."""
    v, t = synth.perturbed_sphere(8, 7)
    G = oracle.slp_dense(v, t, 4)
    touching = np.zeros((len(t), len(t)), dtype=bool)
    for vtx in range(len(v)):
        idx = np.nonzero((t == vtx).any(axis=1))[0]
        touching[np.ix_(idx, idx)] = True
    for m, eps in ((3, 1e-4), (4, 1e-8)):
        A, info = gca.gca_dense(v, t, 16, m, eps, G)
        assert info["far"] > 0
        scale = np.max(np.abs(A))
        D = np.abs(A - A.T)
        assert np.max(D[~touching]) <= 1e-14 * scale, (m, eps)
        assert np.max(D[touching]) <= 1e-5 * scale, (m, eps)
