"""Pins of the oracle's H^2 part (oracle/h2.py) against definitions and
closed forms: cluster and block tree properties (Section 2), admissibility
(Section 3, eq. (admissibility)), Lagrange interpolation identities and the
geometric decay of the interpolation error in the order m (Section 3)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import h2


@pytest.mark.parametrize("space,leaf", [("P0", 8), ("P0", 32), ("P1", 16)])
def test_cluster_tree_definition(space, leaf):
    """Every node is a subset of the index set, the root is the whole set,
    children are disjoint and their union is the parent (Definition "Cluster
    tree"); leaves hold at most ``leaf`` indices and cover contiguous ranges of
    the permutation."""
    v, t = synth.octa_sphere(8)
    pts = v[t].mean(axis=1) if space == "P0" else v
    root, perm, cl = h2.cluster_tree(pts, leaf)
    n = len(pts)
    assert sorted(perm.tolist()) == list(range(n))
    assert root.begin == 0 and root.end == n
    for c in cl:
        assert sorted(c.idx.tolist()) == sorted(perm[c.begin:c.end].tolist())
        if c.children:
            assert len(c.children) == 2
            assert c.children[0].begin == c.begin and c.children[-1].end == c.end
            assert c.children[0].end == c.children[1].begin
            assert not set(c.children[0].idx.tolist()) & set(c.children[1].idx.tolist())
        else:
            assert len(c.idx) <= leaf or np.ptp(pts[c.idx], axis=0).max() == 0


def test_support_boxes_contain_supports():
    v, t = synth.octa_sphere(8)
    root, perm, cl = h2.cluster_tree(v, 16)
    h2.support_boxes(cl, v, t, "P1")
    for c in cl:
        for j in c.idx:
            for tri in t[np.any(t == j, axis=1)]:
                assert np.all(v[tri] >= c.lo - 0) and np.all(v[tri] <= c.hi + 0)


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_block_tree_partitions_the_matrix(kernel):
    """Farfield and nearfield leaves cover I x J exactly once; farfield leaves
    satisfy the admissibility condition, nearfield leaves pair two leaf
    clusters (Definition "Block tree")."""
    v, t = synth.octa_sphere(8)
    cen = v[t].mean(axis=1)
    rt, rp, rcl = h2.cluster_tree(cen, 16)
    h2.support_boxes(rcl, v, t, "P0")
    if kernel == "slp":
        ct, cp, ccl = rt, rp, rcl
        ncol = len(t)
    else:
        ct, cp, ccl = h2.cluster_tree(v, 16)
        h2.support_boxes(ccl, v, t, "P1")
        ncol = len(v)
    far, near = h2.block_tree(rt, ct, 1.0)
    cover = np.zeros((len(t), ncol), dtype=np.int32)
    for (a, b) in far + near:
        cover[a.begin:a.end, b.begin:b.end] += 1
    assert np.all(cover == 1)
    for a, b in far:
        assert max(h2.diam(a), h2.diam(b)) <= 2.0 * h2.dist(a, b)
    for a, b in near:
        assert not a.children and not b.children
    assert len(far) > 0


def test_box_distance_and_diameter_closed_forms():
    class B:
        pass
    a, b = B(), B()
    a.lo, a.hi = np.array([0.0, 0, 0]), np.array([1.0, 2, 2])
    b.lo, b.hi = np.array([4.0, 6, -1]), np.array([5.0, 7, 1])
    assert h2.diam(a) == 3.0
    assert abs(h2.dist(a, b) - 5.0) < 1e-15
    assert h2.dist(a, a) == 0.0


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_lagrange_identities(m):
    """L_nu(xi_mu) = delta, sum_nu L_nu = 1, interpolation reproduces
    polynomials of degree < m per axis, and the gradient of L matches central
    differences."""
    class B:
        pass
    box = B()
    box.lo, box.hi = np.array([-0.3, 0.1, 2.0]), np.array([0.4, 0.9, 2.5])
    ax = h2.box_axes(box, m)
    P = h2.tensor_points(ax)
    L = h2.lagrange_tensor(ax, P)
    np.testing.assert_allclose(L, np.eye(m ** 3), atol=1e-12)
    rng = np.random.default_rng(5)
    X = box.lo + (box.hi - box.lo) * rng.random((20, 3))
    LX = h2.lagrange_tensor(ax, X)
    np.testing.assert_allclose(LX.sum(axis=1), 1.0, atol=1e-12)
    for e in itertools.product(range(m), repeat=3):
        f = lambda Z: Z[:, 0] ** e[0] * Z[:, 1] ** e[1] * Z[:, 2] ** e[2]
        np.testing.assert_allclose(LX @ f(P), f(X), atol=1e-11)
    G = h2.lagrange_tensor_grad(ax, X)
    h = 1e-6
    for d in range(3):
        dX = np.zeros(3)
        dX[d] = h
        fd = (h2.lagrange_tensor(ax, X + dX) - h2.lagrange_tensor(ax, X - dX)) / (2 * h)
        np.testing.assert_allclose(G[:, :, d], fd, atol=1e-6 * max(1.0, np.abs(fd).max()))


def test_leaf_basis_closed_forms():
    """Rows of V_t sum to |tau_i| (partition of unity); for K's column basis,
    applying W_s to the point values of a linear f gives int phi_j df/dn
    = sum_{tau around j} |tau|/3 (a . n_tau) exactly."""
    v, t = synth.octa_sphere(4)
    cen = v[t].mean(axis=1)
    _, _, rcl = h2.cluster_tree(cen, 8)
    h2.support_boxes(rcl, v, t, "P0")
    c = rcl[3]
    ax = h2.box_axes(c, 3)
    V = h2.basis_p0(v, t, c.idx, ax, 7)
    area = 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)
    np.testing.assert_allclose(V.sum(axis=1), area[c.idx], rtol=1e-13)

    _, _, ccl = h2.cluster_tree(v, 4)
    h2.support_boxes(ccl, v, t, "P1")
    s = ccl[5]
    ax = h2.box_axes(s, 3)
    adj = [[] for _ in range(len(v))]
    for k, tri in enumerate(t):
        for j in tri:
            adj[j].append(k)
    W = h2.basis_p1_normal_derivative(v, t, adj, s.idx, ax, 7)
    a = np.array([0.3, -1.1, 0.7])
    fvals = h2.tensor_points(ax) @ a
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    n /= np.linalg.norm(n, axis=1)[:, None]
    expect = np.array([sum(area[k] / 3 * (n[k] @ a) for k in adj[j]) for j in s.idx])
    np.testing.assert_allclose(W @ fvals, expect, atol=1e-13)
    np.testing.assert_allclose(W.sum(axis=1), 0.0, atol=1e-12)


def test_h2_without_farfield_is_the_dense_matrix():
    v, t = synth.octa_sphere(4)
    G = oracle.slp_dense(v, t, 4)
    A, _ = h2.h2_dense(v, t, "slp", 8, 3, near_matrix=G, disable_far=True)
    np.testing.assert_array_equal(A, G)


def test_interpolation_error_decays_geometrically():
    """The interpolation error is bounded by a constant times q^m with q
    depending only on eta (Section 3); in the matrix, the error falls by a
    roughly constant factor per order."""
    v, t = synth.octa_sphere(8)
    G = oracle.slp_dense(v, t, 4)
    errs = []
    for m in (2, 3, 4, 5):
        A, info = h2.h2_dense(v, t, "slp", 16, m, near_matrix=G)
        errs.append(np.linalg.norm(A - G, 2) / np.linalg.norm(G, 2))
    ratios = [errs[i + 1] / errs[i] for i in range(3)]
    assert all(0.02 < r < 0.3 for r in ratios), (errs, ratios)
    assert info["far"] > 0


# ----------------------------------------- sampled rows of the H^2 product

def test_dense_blocks_equal_dense_matrices():
    """Dense entries at chosen rows and columns equal the pinned dense G and K
    (Section 1, eqs. (slp), (dlp)); for K every vertex valence of the mesh is
    among the columns."""
    v, t = synth.perturbed_sphere(4, 401)
    G = oracle.slp_dense(v, t, 4)
    K = oracle.dlp_dense(v, t, 4)
    r = np.array([0, 9, 64, 127])
    c = np.array([5, 0, 127, 64, 64])
    np.testing.assert_allclose(oracle.slp_block(v, t, 4, r, c), G[np.ix_(r, c)], rtol=1e-15, atol=0)
    val = np.bincount(t.ravel(), minlength=len(v))
    cv = np.unique(np.concatenate([[0, len(v) - 1], [np.flatnonzero(val == d)[0] for d in np.unique(val)]]))
    np.testing.assert_allclose(oracle.dlp_block(v, t, 4, r, cv), K[np.ix_(r, cv)], rtol=1e-15, atol=0)


@pytest.mark.parametrize("m", [2, 3])
def test_vectorised_bases_equal_per_triangle_bases(m):
    """The many-triangle forms of the leaf bases (Section 3: integrals of the
    Lagrange polynomials; Section 5: their normal derivatives against the hat
    functions) equal the per-triangle forms."""
    v, t = synth.perturbed_sphere(4, 401)
    cent = v[t].mean(axis=1)
    _, _, cl = h2.cluster_tree(cent, 16)
    h2.support_boxes(cl, v, t, "P0")
    c = cl[3]
    ax = h2.box_axes(c, m)
    idx = np.arange(len(t))[::7]
    np.testing.assert_allclose(h2.basis_p0_many(v, t, idx, ax, 2 * m + 1), h2.basis_p0(v, t, idx, ax, 2 * m + 1),
                               rtol=1e-13, atol=1e-16)
    adj = [[] for _ in range(len(v))]
    for k, tr in enumerate(t):
        for vv in tr:
            adj[vv].append(k)
    vidx = np.arange(len(v))[::5]
    np.testing.assert_allclose(h2.basis_p1_nd_many(v, t, adj, vidx, ax, 2 * m + 1),
                               h2.basis_p1_normal_derivative(v, t, adj, vidx, ax, 2 * m + 1),
                               rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("kernel", ["slp", "dlp"])
def test_h2_rows_equal_dense_h2(kernel):
    """Sampled rows of A X, summed block by block, equal the same rows of the
    written-out H^2 matrix times X (several right-hand sides)."""
    v, t = synth.perturbed_sphere(8, 401)
    A, _ = h2.h2_dense(v, t, kernel, 16, 3)
    X = synth.random_vector(A.shape[1], 6, cols=4).reshape(A.shape[1], 4)
    rows = [0, 13, 255, 300, len(t) - 1]
    Y = h2.h2_rows(v, t, kernel, 16, 3, rows, X)
    ref = A[rows] @ X
    assert np.max(np.abs(Y - ref)) <= 1e-14 * np.max(np.abs(ref))
    y1 = h2.h2_rows(v, t, kernel, 16, 3, rows, X[:, 2])
    assert np.max(np.abs(y1 - ref[:, 2])) <= 1e-14 * np.max(np.abs(ref[:, 2]))


@pytest.mark.parametrize("kernel,m", [("slp", 3), ("dlp", 3), ("slp", 4), ("dlp", 4)])
def test_basis_rule_exact_from_degree(kernel, m):
    """On a flat triangle L_nu is a polynomial of total degree 3(m-1) in the
    reference coordinates (and so is phi_j times a derivative of L_nu), and
    the collapsed q-point rule integrates degree d exactly for
    q >= (d + 2)/2.  So q = (3(m-1) + 3) // 2 gives the same rows as the
    default 2m + 1 points."""
    v, t = synth.perturbed_sphere(8, 401)
    ncol = len(t) if kernel == "slp" else len(v)
    x = synth.random_vector(ncol, 7)
    rows = [3, 100, 400]
    a = h2.h2_rows(v, t, kernel, 16, m, rows, x)
    b = h2.h2_rows(v, t, kernel, 16, m, rows, x, q_basis=(3 * (m - 1) + 3) // 2)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


def _touching(tris):
    """Boolean matrix of the triangle pairs that share a vertex."""
    n = len(tris)
    T = np.zeros((n, n), dtype=bool)
    by_vertex = {}
    for i, tr in enumerate(tris):
        for vtx in tr:
            by_vertex.setdefault(int(vtx), []).append(i)
    for lst in by_vertex.values():
        idx = np.array(lst)
        T[np.ix_(idx, idx)] = True
    return T


def test_single_layer_symmetric_off_touching_pairs():
    """g(x, y) = g(y, x): the Galerkin entries of triangles without a common
    vertex (both orders sum the same tensor Gauss terms) and the interpolation
    far field (kernel values at the same pairs of points, one basis for rows
    and columns) are symmetric to rounding.  Only touching pairs, whose
    singular quadratures differ, break the symmetry, at quadrature error.  G's
    once-per-pair storage of nearfield and far field relies on this."""
    v, t = synth.perturbed_sphere(8, 7)
    G = oracle.slp_dense(v, t, 4)
    A, _ = h2.h2_dense(v, t, "slp", 16, 3, near_matrix=G)
    T = _touching(t)
    for M in (G, A):
        scale = np.max(np.abs(M))
        D = np.abs(M - M.T)
        assert np.max(D[~T]) <= 1e-14 * scale
        assert np.max(D[T]) <= 1e-5 * scale
