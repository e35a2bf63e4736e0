"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of the paper (or the mathematical fact) it checks.
"""
import math

import numpy as np
import pytest

import analytic
import oracle
import synth


def _areas(v, t):
    return 0.5 * np.linalg.norm(np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]]), axis=1)


def _normals(v, t):
    n = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    return n / np.linalg.norm(n, axis=1)[:, None]


# ------------------------------------------------------------ Gauss-Legendre

@pytest.mark.parametrize("q", [1, 2, 3, 5, 8, 13, 20])
def test_gauss_legendre_matches_library_rule(q):
    """The oracle's own Newton-iteration Gauss-Legendre rule equals numpy's."""
    t, w = oracle.gauss_legendre01(q)
    z, wz = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(t, 0.5 * (z + 1.0), rtol=0, atol=1e-14)
    np.testing.assert_allclose(w, 0.5 * wz, rtol=0, atol=1e-14)


@pytest.mark.parametrize("q", [3, 6, 9])
def test_gauss_legendre_exact_for_polynomials(q):
    """q-point rule integrates t^k exactly on [0,1] for k <= 2q-1."""
    t, w = oracle.gauss_legendre01(q)
    for k in range(2 * q):
        assert abs(np.sum(w * t ** k) - 1.0 / (k + 1)) < 1e-14


# ----------------------------------------------- single pairs (brute force)

def _richardson(vals):
    """Extrapolate an O(4^-L) sequence (uniform subdivision of the outer triangle)."""
    a, b = vals[-2], vals[-1]
    return b + (b - a) / 3.0


@pytest.mark.parametrize("kind,angle", [("identical", 0), ("edge", 180), ("edge", 120),
                                        ("edge", 90), ("edge", 60), ("vertex", 0),
                                        ("disjoint", 0)])
def test_slp_pair_against_semianalytic(kind, angle):
    """G_ij of one triangle pair (Section 1, eq. (slp)) equals the reference with
    the inner integral in closed form, for every singular relation that the
    near-field quadrature of Section 5 handles."""
    v, t = synth.single_pair(kind, angle_deg=angle or 120.0)
    tx, ty = v[t[0]], v[t[1]]
    ref = _richardson([analytic.pair_slp_reference(tx, ty, L, 6) for L in (4, 5)])
    val = oracle.slp_entry(v, t, 10, 0, 1)
    assert abs(val - ref) <= 2e-8 * abs(ref)


@pytest.mark.parametrize("kind,angle", [("edge", 120), ("edge", 90), ("edge", 60),
                                        ("vertex", 0), ("disjoint", 0)])
def test_dlp_pair_against_solid_angle(kind, angle):
    """Sum over the three corner weights of a K pair (Section 1, eq. (dlp); the
    barycentric weights add up to one) equals minus the outer integral of the
    triangle's solid angle over 4 pi."""
    v, t = synth.single_pair(kind, angle_deg=angle or 120.0)
    tx, ty = v[t[0]], v[t[1]]
    ref = _richardson([analytic.pair_dlp_constant_reference(tx, ty, L, 6) for L in (4, 5)])
    val = oracle.dlp_pair(v, t, 10, 0, 1).sum()
    assert abs(val - ref) <= 2e-7 * abs(ref)


@pytest.mark.parametrize("kind", ["edge", "vertex"])
def test_singular_rule_converges_exponentially(kind):
    """The regularised rule converges geometrically in q (Section 5 relies on
    raising q_near to keep the convergence rate)."""
    v, t = synth.single_pair(kind)
    vals = [oracle.slp_entry(v, t, q, 0, 1) for q in (3, 5, 7, 9, 11)]
    d = np.abs(np.diff(vals))
    assert np.all(d[1:] < d[:-1] * 0.2)


# ------------------------------------------------------------ whole meshes

def test_gauss_identity_rowwise():
    """Green's formula with u = 1 (Section 1, eq. (green) and its boundary form):
    int_Gamma dg/dn_y(x,y) dy = -1/2 for x in a face of a closed polyhedron, and
    the hat functions sum to one, so (K 1)_i = -|tau_i|/2 row by row.  The
    defect is pure quadrature error and falls as q_near grows."""
    v, t = synth.octa_sphere(4)
    a = _areas(v, t)
    errs = []
    for q in (3, 4, 6):
        K = oracle.dlp_dense(v, t, q)
        errs.append(np.max(np.abs(K.sum(axis=1) / a + 0.5)))
    assert errs[-1] < 2e-6
    assert errs[2] < errs[1] < errs[0]


def test_double_layer_vanishes_on_a_plane():
    """<x - y, n_y> = 0 for coplanar x, y, so K = 0 on a flat mesh."""
    v, t = synth.flat_plate(3)
    K = oracle.dlp_dense(v, t, 4)
    assert np.max(np.abs(K)) < 1e-15


def test_single_layer_symmetry():
    """g(x,y) = g(y,x) makes G symmetric (Section 1, eq. (slp)).  G_ij and G_ji
    are computed independently (roles of the two triangles swapped): disjoint
    pairs agree to rounding, touching pairs to quadrature error."""
    v, t = synth.octa_sphere(4)
    G = oracle.slp_dense(v, t, 5)
    shared = np.array([[len(set(t[i]) & set(t[j])) for j in range(len(t))] for i in range(len(t))])
    D = np.abs(G - G.T) / np.abs(G).max()
    assert D[shared == 0].max() < 1e-14
    assert D[shared > 0].max() < 1e-6


def test_octahedron_entry_classes():
    """On the regular octahedron (s = 1) all faces are congruent, so G has one
    value per relation class: identical, common edge, common vertex, opposite."""
    v, t = synth.octa_sphere(1)
    G = oracle.slp_dense(v, t, 8)
    classes = {}
    for i in range(8):
        for j in range(8):
            ns = len(set(t[i]) & set(t[j]))
            if ns == 0:
                # disjoint faces of an octahedron are either opposite or share nothing but are adjacent by a vertex pair
                key = ("opp", round(float(np.linalg.norm(v[t[i]].mean(0) + v[t[j]].mean(0))), 6))
            else:
                key = ns
            classes.setdefault(key, []).append(G[i, j])
    for key, vals in classes.items():
        vals = np.array(vals)
        assert np.ptp(vals) <= 1e-8 * np.abs(vals).max(), key
    assert len(classes) == 4


@pytest.mark.parametrize("l,poly", [
    (0, lambda p: np.ones(len(p))),
    (1, lambda p: p[:, 0]),
    (2, lambda p: p[:, 0] * p[:, 1]),
    (3, lambda p: p[:, 0] * p[:, 1] * p[:, 2]),
    (4, lambda p: p[:, 0] ** 4 - 6 * p[:, 0] ** 2 * p[:, 1] ** 2 + p[:, 1] ** 4),
])
def test_single_layer_sphere_spectrum(l, poly):
    """On the unit sphere the single-layer operator maps a degree-l spherical
    harmonic Y to Y/(2l+1) (classical; the kernel g is the one of Section 1).
    The Galerkin Rayleigh quotient c^T G c / c^T D c, D = diag|tau_i|, tends to
    1/(2l+1) as the octahedral mesh of Section 5 is refined."""
    errs = []
    for s in (4, 8, 16):
        v, t = synth.octa_sphere(s)
        cen = v[t].mean(axis=1)
        c = poly(cen / np.linalg.norm(cen, axis=1)[:, None])
        G = oracle.slp_dense(v, t, 4)
        R = c @ G @ c / np.sum(c * c * _areas(v, t))
        errs.append(abs(R - 1.0 / (2 * l + 1)))
    assert errs[0] > errs[1] > errs[2]
    rate = math.log2(errs[1] / errs[2])
    assert rate > 1.5, (errs, rate)
    assert errs[2] < 0.02 / (2 * l + 1)


def _mass(v, t):
    M = np.zeros((len(t), len(v)))
    a = _areas(v, t)
    for i, tri in enumerate(t):
        for c in tri:
            M[i, c] += a[i] / 3.0
    return M


@pytest.mark.parametrize("a,b", [((1.0, 0.0, 0.0), 0.0), ((0.3, -0.7, 0.5), 1.3)])
def test_discrete_green_identity_linear(a, b):
    """Green's boundary formula (Section 1) tested with psi_i gives
    G (du/dn) = (M/2 + K) u, the Dirichlet-to-Neumann system of eq.
    (matrix_dtn).  For a linear (harmonic) u on the flat mesh, u is exactly its
    P1 interpolant and du/dn = a . n_tau exactly in P0, and the formula holds on
    a closed polyhedron; the residual is quadrature error only."""
    v, t = synth.octa_sphere(4)
    a = np.array(a)
    u = v @ a + b
    dudn = _normals(v, t) @ a
    q = 6
    G = oracle.slp_dense(v, t, q)
    K = oracle.dlp_dense(v, t, q)
    lhs = G @ dudn
    rhs = (0.5 * _mass(v, t) + K) @ u
    scale = np.abs(0.5 * _mass(v, t) @ u).max() + np.abs(lhs).max()
    assert np.max(np.abs(lhs - rhs)) < 1e-6 * scale


def test_discrete_green_identity_paper_functions_converge():
    """The paper's test functions u1 = x1^2 - x3^2 and u2 = g(., y1), y1 =
    (1.2,1.2,1.2) (Section 5), harmonic inside the unit sphere.  Their P1
    interpolants and P0 projections of du/dn satisfy G q = (M/2 + K) u only up to
    discretisation error, which falls as the mesh is refined."""
    y1 = np.array([1.2, 1.2, 1.2])

    def u1(p):
        return p[:, 0] ** 2 - p[:, 2] ** 2

    def du1(p, n):
        return 2 * p[:, 0] * n[:, 0] - 2 * p[:, 2] * n[:, 2]

    def u2(p):
        return 1.0 / (4 * math.pi * np.linalg.norm(p - y1, axis=1))

    def du2(p, n):
        d = p - y1
        r = np.linalg.norm(d, axis=1)
        return -np.einsum("ij,ij->i", d, n) / (4 * math.pi * r ** 3)

    for u, du in ((u1, du1), (u2, du2)):
        res = []
        for s in (2, 4, 8):
            v, t = synth.octa_sphere(s)
            n = _normals(v, t)
            rule_u = np.array([[1 / 6, 1 / 6, 2 / 3], [1 / 6, 2 / 3, 1 / 6], [2 / 3, 1 / 6, 1 / 6]])
            # P0 L2-projection of du/dn by a degree-2-exact triangle rule
            P = np.einsum("kc,icd->ikd", rule_u, v[t])
            q0 = np.mean([du(P[:, k, :], n) for k in range(3)], axis=0)
            G = oracle.slp_dense(v, t, 5)
            K = oracle.dlp_dense(v, t, 5)
            r = G @ q0 - (0.5 * _mass(v, t) + K) @ u(v)
            res.append(np.linalg.norm(r) / np.linalg.norm(0.5 * _mass(v, t) @ u(v)))
        assert res[0] > res[1] > res[2], res


# ------------------------------------------------ sampled rows of the products

@pytest.mark.parametrize("trans", [False, True])
def test_slp_rows_equal_dense_matrix(trans):
    """The sampled rows of G x and G^T x (Section 1, eq. (slp)) that every
    large-mesh check uses equal rows and columns of the dense matrix, which the
    pins above tie to closed forms.  A perturbed sphere has no symmetry, so a
    swapped index (row for column) would show."""
    v, t = synth.perturbed_sphere(4, 401)
    G = oracle.slp_dense(v, t, 4)
    x = synth.random_vector(len(t), 21)
    rows = np.array([0, 5, 17, 63, 64, 100, len(t) - 1])
    y = oracle.slp_rows(v, t, 4, rows, x, trans=trans)
    ref = (G.T if trans else G)[rows] @ x
    np.testing.assert_allclose(y, ref, rtol=1e-14, atol=1e-14 * np.max(np.abs(ref)))


@pytest.mark.parametrize("trans", [False, True])
def test_dlp_rows_equal_dense_matrix(trans):
    """Rows of K x (triangles) and of K^T x (vertices; the pair contributions
    summed over the triangles around each vertex, Section 1, eq. (dlp)) equal
    rows and columns of the dense K, pinned by Gauss's identity and the flat
    plate.  The transposed branch looks up each vertex's corner slot on its own,
    so it is checked at vertices of every valence the mesh has."""
    v, t = synth.perturbed_sphere(4, 401)
    K = oracle.dlp_dense(v, t, 4)
    x = synth.random_vector(len(t) if trans else len(v), 22)
    if trans:
        valence = np.bincount(t.ravel(), minlength=len(v))
        rows = np.unique(np.concatenate([[0, len(v) - 1],
                                         [np.flatnonzero(valence == d)[0] for d in np.unique(valence)]]))
        ref = K[:, rows].T @ x
    else:
        rows = np.array([0, 3, 31, 64, 99, len(t) - 1])
        ref = K[rows] @ x
    y = oracle.dlp_rows(v, t, 4, rows, x, trans=trans)
    np.testing.assert_allclose(y, ref, rtol=1e-14, atol=1e-14 * np.max(np.abs(ref)))
