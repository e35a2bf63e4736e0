"""Pins of the oracle's mass matrix, conjugate gradient method,
Dirichlet-to-Neumann solve, hypersingular matrix and Neumann-to-Dirichlet
solve against facts that do not come from the oracle itself: exact
integration of linear functions, finite termination and the energy-norm
optimality of CG, closed-form Neumann data of harmonic functions, the
eigenvalues of the hypersingular operator on the sphere, and the L2
convergence orders that Section 5 states (O(h) for the Neumann data, O(h^2)
for the Dirichlet data)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import krylov


def _geom(v, t):
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(b - a, c - a)
    nrm = np.linalg.norm(cr, axis=1)
    return 0.5 * nrm, cr / nrm[:, None], (a + b + c) / 3.0


# ---------------------------------------------------------------- mass matrix

@pytest.mark.parametrize("mesh", ["sphere", "ellipsoid", "perturbed"])
def test_mass_matrix_integrates_linear_functions_exactly(mesh):
    """Sum_j m_ij = |tau_i| (the hat functions sum to one) and
    Sum_j m_ij x_j = |tau_i| * centroid (a linear function equals its P1
    interpolant, and the mean of a linear function over a triangle is its
    value at the centroid).  Four equations for the three corner entries of a
    row: together they fix M."""
    if mesh == "sphere":
        v, t = synth.octa_sphere(4)
    elif mesh == "ellipsoid":
        v, t = synth.ellipsoid(4, 0.7, 1.3, 2.1)
    else:
        v, t = synth.perturbed_sphere(4, seed=7)
    M = krylov.mass_matrix(v, t)
    area, _, cen = _geom(v, t)
    assert np.allclose(M.sum(axis=1), area, rtol=1e-14, atol=0)
    for d in range(3):
        assert np.allclose(M @ v[:, d], area * cen[:, d], rtol=1e-12, atol=1e-15)
    assert np.count_nonzero(M) == 3 * len(t)


# ---------------------------------------------------------- conjugate gradients

def _spd(n, eigs, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * eigs) @ Q.T


def test_cg_matches_direct_solve():
    """On a random SPD matrix (condition 1e3) CG converges to the solution of
    numpy's dense solver."""
    n = 40
    A = _spd(n, np.geomspace(1.0, 1e3, n), 1)
    b = np.random.default_rng(2).standard_normal(n)
    x, k, hist = krylov.cg(lambda p: A @ p, b, 1e-13, 500)
    assert hist[-1] <= 1e-13 and k < 500
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)


def test_cg_terminates_after_as_many_steps_as_distinct_eigenvalues():
    """In exact arithmetic CG finds the solution after at most as many steps
    as A has distinct eigenvalues (three here, each of multiplicity ten); a
    wrong step length or direction update loses this."""
    A = _spd(30, np.repeat([1.0, 3.0, 10.0], 10), 3)
    b = np.random.default_rng(4).standard_normal(30)
    x, k, hist = krylov.cg(lambda p: A @ p, b, 1e-10, 100)
    assert k == 3, hist
    assert hist[2] > 1e-3
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_cg_iterate_minimises_the_energy_norm_over_the_krylov_space(k):
    """The k-th CG iterate is the minimiser of ||x* - x||_A over x0 + K_k(A, r0)
    (the Galerkin solution on the Krylov space), computed here independently
    from an orthonormal basis of span{r0, A r0, ..., A^{k-1} r0}."""
    n = 25
    A = _spd(n, np.geomspace(1.0, 50.0, n), 5)
    rng = np.random.default_rng(6)
    b, x0 = rng.standard_normal(n), rng.standard_normal(n)
    x, it, hist = krylov.cg(lambda p: A @ p, b, 0.0, k, x0=x0)
    assert it == k
    r0 = b - A @ x0
    kry = [r0]
    for _ in range(k - 1):
        kry.append(A @ kry[-1])
    Q, _ = np.linalg.qr(np.array(kry).T)
    y = np.linalg.solve(Q.T @ A @ Q, Q.T @ r0)
    xg = x0 + Q @ y
    assert np.linalg.norm(x - xg) <= 1e-9 * np.linalg.norm(xg)
    # the recurrence residual is the true residual
    assert abs(np.linalg.norm(b - A @ x) / np.linalg.norm(b) - hist[-1]) <= 1e-10


def test_cg_stopping_rule_and_degenerate_cases():
    A = _spd(20, np.geomspace(1.0, 100.0, 20), 8)
    b = np.random.default_rng(9).standard_normal(20)
    x, k, hist = krylov.cg(lambda p: A @ p, b, 1e-6, 100)
    assert hist[k] <= 1e-6 < hist[k - 1]
    assert len(hist) == k + 1 and hist[0] == pytest.approx(1.0)
    # no iterations: the initial guess comes back
    x0 = np.arange(20.0)
    x, k, hist = krylov.cg(lambda p: A @ p, b, 1e-6, 0, x0=x0)
    assert k == 0 and np.array_equal(x, x0)
    # b = 0 from the zero guess: solved before the first step
    x, k, hist = krylov.cg(lambda p: A @ p, np.zeros(20), 1e-6, 10)
    assert k == 0 and not x.any()


def test_pcg_limits():
    """Preconditioned CG: with the identity it is CG step for step; with the
    exact inverse it converges in one step; with block-Jacobi on a
    block-diagonal SPD matrix it converges in one step."""
    n = 24
    A = _spd(n, np.geomspace(1.0, 100.0, n), 12)
    b = np.random.default_rng(13).standard_normal(n)
    x0, k0, h0 = krylov.cg(lambda p: A @ p, b, 1e-10, 200)
    x1, k1, h1 = krylov.pcg(lambda p: A @ p, lambda r: r.copy(), b, 1e-10, 200)
    assert k0 == k1 and np.allclose(h0, h1, rtol=1e-9, atol=0)
    Ai = np.linalg.inv(A)
    _, k2, _ = krylov.pcg(lambda p: A @ p, lambda r: Ai @ r, b, 1e-10, 200)
    assert k2 == 1
    blocks = [np.arange(0, 10), np.arange(10, 16), np.arange(16, 24)]
    D = np.zeros((n, n))
    for idx in blocks:
        D[np.ix_(idx, idx)] = _spd(len(idx), np.geomspace(1.0, 30.0, len(idx)), 20 + len(idx))
    _, k3, _ = krylov.pcg(lambda p: D @ p, krylov.block_jacobi(D, blocks), b, 1e-10, 200)
    assert k3 == 1


# ----------------------------------------------------- Dirichlet-to-Neumann

def test_l2_error_of_exact_and_shifted_data():
    """For linear u the normal derivative is the constant a . n_tau on each
    flat triangle: the error of that P0 function is zero, and shifting it by
    delta gives delta * sqrt(|Gamma|)."""
    v, t = synth.octa_sphere(4)
    area, n, _ = _geom(v, t)
    a = np.array([0.3, -0.8, 0.5])
    grad = lambda p: np.broadcast_to(a, p.shape)  # noqa: E731
    assert krylov.neumann_l2_error(v, t, n @ a, grad) <= 1e-14
    d = 0.125
    assert krylov.neumann_l2_error(v, t, n @ a + d, grad) == pytest.approx(d * math.sqrt(area.sum()), rel=1e-12)


def test_dtn_reproduces_linear_neumann_data():
    """Green's formula (Section 1) holds exactly on the polyhedron for a
    linear u, which is its own P1 interpolant and has P0 Neumann data
    a . n_tau; the solution of eq. (matrix_dtn) differs from that only by
    quadrature error, which falls exponentially with the order q."""
    v, t = synth.octa_sphere(4)
    _, n, _ = _geom(v, t)
    a = np.array([1.0, -0.5, 0.25])
    err = []
    for q in (4, 8, 12):
        G, K, M = krylov.dtn_matrices(v, t, q)
        sol = krylov.dtn_solve(G, K, M, v @ a + 0.7)
        err.append(np.max(np.abs(sol - n @ a)) / np.max(np.abs(n @ a)))
    assert err[0] > 100 * err[1] > 1e4 * err[2], err
    assert err[2] <= 1e-9, err


def test_dtn_paper_functions_converge_first_order():
    """Section 5: the Neumann data of u1, u2 and u3 computed from eq.
    (matrix_dtn) converge in L2 at the rate O(h).  The observed order between
    the two finest meshes (s = 8 and 16, h halved) is checked for each."""
    errs = {name: [] for name in krylov.TEST_FUNCTIONS}
    for s in (4, 8, 16):
        v, t = synth.octa_sphere(s)
        G, K, M = krylov.dtn_matrices(v, t, 4)
        for name, (u, grad) in krylov.TEST_FUNCTIONS.items():
            sol = krylov.dtn_solve(G, K, M, u(v))
            errs[name].append(krylov.neumann_l2_error(v, t, sol, grad))
    for name, e in errs.items():
        assert e[0] > e[1] > e[2], (name, e)
        rate = math.log2(e[1] / e[2])
        assert 0.8 <= rate <= 1.6, (name, e, rate)


# ------------------------------------------------ hypersingular, Neumann-to-Dirichlet

def test_surface_curls_of_linear_functions():
    """On a flat triangle the surface curl n x grad_Gamma u of u = a . x is
    n_tau x a, and constants have zero curl; three components per triangle
    fix the three corner entries of each row of C_d."""
    v, t = synth.perturbed_sphere(4, seed=5)
    _, n, _ = _geom(v, t)
    C = krylov.curl_matrices(v, t)
    a = np.array([0.3, -0.8, 0.5])
    got = np.stack([C[d] @ (v @ a) for d in range(3)], axis=1)
    assert np.max(np.abs(got - np.cross(n, a))) <= 1e-13
    assert np.max(np.abs(np.stack([C[d] @ np.ones(len(v)) for d in range(3)]))) <= 1e-13
    b = np.array([-0.1, 0.4, 0.9])
    got = np.stack([C[d] @ (v @ b) for d in range(3)], axis=1)
    assert np.max(np.abs(got - np.cross(n, b))) <= 1e-13


def test_hypersingular_spectrum_on_the_sphere():
    """The hypersingular operator of the unit sphere has the spherical
    harmonics of degree l as eigenfunctions with eigenvalue l(l+1)/(2l+1)
    (classical; not printed in the paper).  Rayleigh quotients of the P1
    interpolants of degree-1, 2 and 3 harmonics approach it at second order,
    and W annihilates constants."""
    harmonics = ((1, lambda p: p[:, 2]), (2, lambda p: p[:, 0] * p[:, 1]), (3, lambda p: p[:, 0] * p[:, 1] * p[:, 2]))
    rel = []
    for s in (4, 8):
        v, t = synth.octa_sphere(s)
        W = krylov.hypersingular_from_slp(oracle.slp_dense(v, t, 4), krylov.curl_matrices(v, t))
        M1 = krylov.p1_mass_matrix(v, t)
        assert np.max(np.abs(W @ np.ones(len(v)))) <= 1e-14 * np.max(np.abs(W))
        row = []
        for l, f in harmonics:
            c = f(v)
            row.append(abs((c @ W @ c) / (c @ M1 @ c) / (l * (l + 1) / (2 * l + 1)) - 1))
        rel.append(row)
    for l in range(3):
        assert rel[1][l] < 0.015 and rel[0][l] / rel[1][l] > 3.0, rel


def test_ntd_reproduces_linear_dirichlet_data():
    """For linear u the Neumann data a . n_tau are exact in P0 and u is its
    own P1 interpolant; the hypersingular equation of Green's formula holds
    on the polyhedron, so the solution of eq. (matrix_ntd) with zero mean is
    the zero-mean nodal u up to quadrature error, falling exponentially in q."""
    v, t = synth.octa_sphere(4)
    _, n, _ = _geom(v, t)
    a = np.array([1.0, -0.5, 0.25])
    err = []
    for q in (4, 8, 12):
        G, K, M = krylov.dtn_matrices(v, t, q)
        W = krylov.hypersingular_from_slp(G, krylov.curl_matrices(v, t))
        u = krylov.ntd_solve(W, K, M, n @ a)
        ex = v @ a
        w1 = M.sum(axis=0)
        ex = ex - (w1 @ ex) / w1.sum()
        err.append(np.max(np.abs(u - ex)) / np.max(np.abs(ex)))
    assert err[0] > 100 * err[1] > 1e4 * err[2], err
    assert err[2] <= 1e-10, err


def test_ntd_paper_functions_converge_second_order():
    """Section 5: the Dirichlet data of u1, u2, u3 computed from eq.
    (matrix_ntd) with the P0 projection of their Neumann data converge in L2
    at O(h^2) (observed order between s = 8 and 16)."""
    errs = {name: [] for name in krylov.TEST_FUNCTIONS}
    for s in (4, 8, 16):
        v, t = synth.octa_sphere(s)
        G, K, M = krylov.dtn_matrices(v, t, 4)
        W = krylov.hypersingular_from_slp(G, krylov.curl_matrices(v, t))
        for name, (u, grad) in krylov.TEST_FUNCTIONS.items():
            uh = krylov.ntd_solve(W, K, M, krylov.neumann_projection(v, t, grad))
            errs[name].append(krylov.dirichlet_l2_error(v, t, uh, u))
    for name, e in errs.items():
        assert e[0] > e[1] > e[2], (name, e)
        rate = math.log2(e[1] / e[2])
        assert 1.7 <= rate <= 2.5, (name, e, rate)


def test_error_measures_of_exact_data():
    """The measuring sticks of the convergence tests: a linear function is its
    own P1 interpolant, so its Dirichlet L2 error is zero for any added
    constant, and a constant shift of a P1 function does not change the
    zero-mean error; the P0 projection of the normal derivative of a linear
    function is a . n_tau exactly; for u1 the Dirichlet error of the nodal
    interpolant falls at second order."""
    v, t = synth.perturbed_sphere(4, seed=9)
    _, n, _ = _geom(v, t)
    a = np.array([0.2, -1.1, 0.7])
    lin = lambda p: p @ a  # noqa: E731
    assert krylov.dirichlet_l2_error(v, t, v @ a + 5.0, lin) <= 1e-13
    grad = lambda p: np.broadcast_to(a, p.shape)  # noqa: E731
    assert np.max(np.abs(krylov.neumann_projection(v, t, grad) - n @ a)) <= 1e-14
    rng = np.random.default_rng(4)
    uh = krylov.u1(v) + 0.01 * rng.standard_normal(len(v))
    e0 = krylov.dirichlet_l2_error(v, t, uh, krylov.u1)
    assert krylov.dirichlet_l2_error(v, t, uh + 3.0, krylov.u1) == pytest.approx(e0, rel=1e-12)
    errs = []
    for s in (4, 8, 16):
        vs, ts = synth.octa_sphere(s)
        errs.append(krylov.dirichlet_l2_error(vs, ts, krylov.u1(vs), krylov.u1))
    assert 1.7 <= math.log2(errs[1] / errs[2]) <= 2.3, errs


def test_energy_norm_of_constants_and_exact_data():
    """The G-norm: on the unit sphere the single-layer potential of the
    constant density 1 is 1, so 1^T G 1 tends to |S| = 4 pi (the polyhedral
    mesh misses it by O(h^2): the gap shrinks about fourfold as h halves);
    the norm is absolutely homogeneous; the energy error of the exact P0
    Neumann data of a linear function is zero."""
    gaps = []
    for s in (4, 8, 16):
        v, t = synth.octa_sphere(s)
        G = oracle.slp_dense(v, t, 4)
        gaps.append(abs(krylov.energy_norm(G, np.ones(len(t))) ** 2 - 4.0 * math.pi))
    assert gaps[0] > gaps[1] > gaps[2]
    assert 3.0 <= gaps[1] / gaps[2] <= 5.0, gaps
    v, t = synth.perturbed_sphere(4, seed=6)
    G = oracle.slp_dense(v, t, 4)
    e = synth.random_vector(len(t), 8)
    assert krylov.energy_norm(G, -2.5 * e) == pytest.approx(2.5 * krylov.energy_norm(G, e), rel=1e-13)
    _, n, _ = _geom(v, t)
    a = np.array([0.4, 0.9, -0.3])
    grad = lambda p: np.broadcast_to(a, p.shape)  # noqa: E731
    assert krylov.neumann_energy_error(G, v, t, n @ a, grad) <= 1e-12


def test_dtn_energy_error_converges_second_order():
    """Section 5: the discrete H^{-1/2} error (G-norm of the difference between
    the P0 projection of the exact Neumann data and the Galerkin solution of
    eq. (matrix_dtn)) falls like O(h^2) for u1, u2 and u3; the observed order
    between s = 8 and 16 is checked."""
    errs = {name: [] for name in krylov.TEST_FUNCTIONS}
    for s in (8, 16):
        v, t = synth.octa_sphere(s)
        G, K, M = krylov.dtn_matrices(v, t, 4)
        for name, (u, grad) in krylov.TEST_FUNCTIONS.items():
            sol = krylov.dtn_solve(G, K, M, u(v))
            errs[name].append(krylov.neumann_energy_error(G, v, t, sol, grad))
    for name, e in errs.items():
        rate = math.log2(e[0] / e[1])
        assert 1.6 <= rate <= 2.8, (name, e, rate)
