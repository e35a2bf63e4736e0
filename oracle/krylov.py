"""Test infrastructure only: the Dirichlet-to-Neumann and Neumann-to-Dirichlet
systems and the conjugate gradient method, dense and in double precision
(small meshes only).

* Mixed mass matrix (Section 1): m_ij = int psi_i phi_j for the piecewise
  constant psi_i (triangles) and the piecewise linear hat functions phi_j
  (vertices).  On a flat triangle the hat function of one of its corners
  integrates to a third of the area, so m_ij = |tau_i| / 3 when j is a corner
  of tau_i and 0 otherwise.
* Dirichlet-to-Neumann system (Section 1, eq. (matrix_dtn)): G t = (M/2 + K) u
  for the Neumann coefficients t given the Dirichlet coefficients u.  Its
  exact solution is the plain definition G^{-1} (M/2 + K) u, computed here by
  a dense direct solve.
* Conjugate gradients (Hestenes and Stiefel, 1952), the Krylov solver the
  experiments of Section 5 run on this system with relative accuracy
  eps_slv: stop at the first iterate whose residual satisfies
  ||b - A x_k||_2 <= tol ||b||_2, where the residual is the one the
  recurrence updates.
* Hypersingular matrix (Section 1, eq. for w_ij, set up through the
  alternative representation based on the single-layer operator that the
  paper cites): for the hat functions on flat triangles,
  w_ij = sum over triangle pairs of <curl phi_i|tau, curl phi_j|tau'> g_{tau tau'},
  with g_{tau tau'} the single-layer entries of the triangle indicators and
  the surface curl n x grad phi constant on each triangle; on tau with
  corners (a, b, c) in counter-clockwise order, curl phi_a = (x_b - x_c) / (2|tau|)
  and cyclically.  So W = sum_d C_d^T G C_d with (C_d)_{tau j} the d-th
  component of curl phi_j on tau.
* Neumann-to-Dirichlet system (Section 1, eq. (matrix_ntd)):
  W u = (M^T/2 - K^T) t.  W annihilates constants, so the discrete Dirichlet
  data are fixed up to a constant; the direct solve here picks the solution
  with int u_h = 0 (an added Lagrange multiplier).
* Discrete H^{-1/2} error of the Neumann data (Section 5, the energy-norm
  error the experiments report beside the L2 error): for the P0 L2
  projection Pi t of the exact normal derivative and the computed t_h, the
  single-layer operator defines the norm, ||e||_G = sqrt(e^T G e) with
  e = Pi t - t_h.  A plain matrix form; G is symmetric positive definite.
* The test functions of Section 5: u1(x) = x1^2 - x3^2, u2 = g(., y1) and
  u3 = g(., y2) with y1 = (1.2, 1.2, 1.2), y2 = (1.0, 0.25, 1.0), all
  harmonic inside the unit sphere, and the L2 error of a piecewise constant
  Neumann approximation against the exact normal derivative <grad u, n_tau>
  on the flat triangles of the mesh.
"""
import math

import numpy as np

from . import slp_dense, dlp_dense
from .h2 import triangle_rule

FOUR_PI = 4.0 * math.pi
Y1 = np.array([1.2, 1.2, 1.2])
Y2 = np.array([1.0, 0.25, 1.0])


def _areas_normals(verts, tris):
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(b - a, c - a)
    nrm = np.linalg.norm(cr, axis=1)
    return 0.5 * nrm, cr / nrm[:, None]


def mass_matrix(verts, tris):
    """Dense mixed mass matrix M (nt x nv), m_ij = |tau_i| / 3 for the
    corners j of tau_i."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    area, _ = _areas_normals(verts, tris)
    M = np.zeros((len(tris), len(verts)))
    for i in range(len(tris)):
        for j in tris[i]:
            M[i, j] += area[i] / 3.0
    return M


def cg(apply_a, b, tol, max_iter, x0=None):
    """Conjugate gradients for a symmetric positive definite operator.

    Returns (x, iterations, history) where history[k] = ||r_k|| / ||b|| for
    the recurrence residuals r_0 .. r_iterations (the absolute norm when
    b = 0).  Stops at the first k with ||r_k|| <= tol ||b||, or after
    max_iter iterations, or when p^T A p is not positive (breakdown)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - apply_a(x) if x0 is not None else b.copy()
    bnorm = math.sqrt(float(b @ b))
    scale = bnorm if bnorm > 0 else 1.0
    rho = float(r @ r)
    history = [math.sqrt(rho) / scale]
    p = r.copy()
    k = 0
    while math.sqrt(rho) > tol * bnorm and k < max_iter:
        q = apply_a(p)
        pq = float(p @ q)
        if not pq > 0:
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rho_new = float(r @ r)
        beta = rho_new / rho
        rho = rho_new
        p = r + beta * p
        k += 1
        history.append(math.sqrt(rho) / scale)
    return x, k, np.array(history)


def pcg(apply_a, apply_m, b, tol, max_iter):
    """Preconditioned conjugate gradients from x = 0 with the symmetric
    positive definite preconditioner z = apply_m(r): rho = r^T z, the same
    stopping rule on ||r|| as cg().  Returns (x, iterations, history)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = math.sqrt(float(b @ b))
    scale = bnorm if bnorm > 0 else 1.0
    z = apply_m(r)
    rho = float(r @ z)
    p = z.copy()
    history = [math.sqrt(float(r @ r)) / scale]
    k = 0
    while history[-1] * scale > tol * bnorm and k < max_iter:
        q = apply_a(p)
        pq = float(p @ q)
        if not pq > 0:
            break
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        z = apply_m(r)
        rho_new = float(r @ z)
        p = z + (rho_new / rho) * p
        rho = rho_new
        k += 1
        history.append(math.sqrt(float(r @ r)) / scale)
    return x, k, np.array(history)


def block_jacobi(A, blocks):
    """Block-diagonal preconditioner: the inverses of the symmetric parts of
    the diagonal blocks A[idx, idx] for the index lists `blocks`, returned as
    a function r -> z."""
    inv = []
    for idx in blocks:
        B = A[np.ix_(idx, idx)]
        inv.append((idx, np.linalg.inv(0.5 * (B + B.T))))

    def apply(r):
        z = np.zeros_like(r)
        for idx, Bi in inv:
            z[idx] = Bi @ r[idx]
        return z

    return apply


def dtn_matrices(verts, tris, q):
    """Dense G, K and M of one mesh (nearfield quadrature order q everywhere)."""
    return slp_dense(verts, tris, q), dlp_dense(verts, tris, q), mass_matrix(verts, tris)


def dtn_rhs(K, M, u):
    """Right-hand side (M/2 + K) u of eq. (matrix_dtn)."""
    return 0.5 * (M @ u) + K @ u


def dtn_solve(G, K, M, u):
    """Neumann coefficients t = G^{-1} (M/2 + K) u by a dense direct solve."""
    return np.linalg.solve(G, dtn_rhs(K, M, u))


# ------------------------------------------------------- test functions

def u1(p):
    return p[..., 0] ** 2 - p[..., 2] ** 2


def grad_u1(p):
    g = np.zeros_like(p)
    g[..., 0] = 2.0 * p[..., 0]
    g[..., 2] = -2.0 * p[..., 2]
    return g


def _point_source(y):
    def u(p):
        return 1.0 / (FOUR_PI * np.linalg.norm(p - y, axis=-1))

    def grad(p):
        d = p - y
        r = np.linalg.norm(d, axis=-1)
        return -d / (FOUR_PI * r ** 3)[..., None]

    return u, grad


u2, grad_u2 = _point_source(Y1)
u3, grad_u3 = _point_source(Y2)
TEST_FUNCTIONS = {"u1": (u1, grad_u1), "u2": (u2, grad_u2), "u3": (u3, grad_u3)}


def neumann_l2_error(verts, tris, t, grad_u, q=6):
    """|| t - <grad u, n_tau> ||_{L2(Gamma)} for the piecewise constant t,
    integrated with the collapsed q x q Gauss rule on every triangle."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    area, n = _areas_normals(verts, tris)
    U, W = triangle_rule(q)
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    # x(u1, u2) = a + u1 (b - a) + u2 (c - b); the rule integrates over the
    # reference triangle of area 1/2, so the Jacobian is 2 |tau|
    X = a[:, None, :] + U[None, :, :1] * (b - a)[:, None, :] + U[None, :, 1:2] * (c - b)[:, None, :]
    dn = np.einsum("ikd,id->ik", grad_u(X), n)
    err2 = np.einsum("ik,k,i->", (t[:, None] - dn) ** 2, W, 2.0 * area)
    return math.sqrt(err2)


# ------------------------------------------------ hypersingular operator

def curl_matrices(verts, tris):
    """Dense C_0, C_1, C_2 (nt x nv each): (C_d)_{tau j} = d-th component of
    the surface curl of the hat function phi_j on triangle tau."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    area, _ = _areas_normals(verts, tris)
    C = np.zeros((3, len(tris), len(verts)))
    for i, (a, b, c) in enumerate(tris):
        for j, nxt, prv in ((a, b, c), (b, c, a), (c, a, b)):
            C[:, i, j] += (verts[nxt] - verts[prv]) / (2.0 * area[i])
    return C


def hypersingular_from_slp(G, C):
    """W = sum_d C_d^T G C_d."""
    return sum(C[d].T @ G @ C[d] for d in range(3))


def p1_mass_matrix(verts, tris):
    """int phi_i phi_j: |tau|/6 on the diagonal and |tau|/12 off it, per triangle."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    area, _ = _areas_normals(verts, tris)
    M1 = np.zeros((len(verts), len(verts)))
    for i, tri in enumerate(tris):
        for a in tri:
            for b in tri:
                M1[a, b] += area[i] / (6.0 if a == b else 12.0)
    return M1


def ntd_rhs(K, M, t):
    """Right-hand side (M^T/2 - K^T) t of eq. (matrix_ntd)."""
    return 0.5 * (M.T @ t) - K.T @ t


def ntd_solve(W, K, M, t):
    """Dirichlet coefficients u with W u = (M^T/2 - K^T) t and int u_h = 0
    (dense direct solve of the system bordered by the P1 integrals)."""
    w1 = M.sum(axis=0)  # int phi_j
    n = W.shape[0]
    A = np.zeros((n + 1, n + 1))
    A[:n, :n] = W
    A[:n, n] = w1
    A[n, :n] = w1
    rhs = np.concatenate([ntd_rhs(K, M, t), [0.0]])
    return np.linalg.solve(A, rhs)[:n]


def dirichlet_l2_error(verts, tris, uh, u, q=6):
    """|| (u_h - mean u_h) - (u - mean u) ||_{L2(Gamma)} for the P1 function
    u_h (vertex coefficients) against the function u on the flat triangles
    (both taken with zero mean: the Neumann data fix u only up to a constant)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    area, _ = _areas_normals(verts, tris)
    U, W = triangle_rule(q)
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    X = a[:, None, :] + U[None, :, :1] * (b - a)[:, None, :] + U[None, :, 1:2] * (c - b)[:, None, :]
    # barycentric weights of x = a + u1 (b - a) + u2 (c - b): (1 - u1, u1 - u2, u2)
    lam = np.stack([1.0 - U[:, 0], U[:, 0] - U[:, 1], U[:, 1]], axis=1)
    vh = np.einsum("kc,ic->ik", lam, uh[tris])
    vu = u(X)
    wts = W[None, :] * (2.0 * area)[:, None]
    tot = wts.sum()
    d = (vh - (vh * wts).sum() / tot) - (vu - (vu * wts).sum() / tot)
    return math.sqrt(float((d * d * wts).sum()))


def neumann_projection(verts, tris, grad_u, q=6):
    """P0 L2 projection of the normal derivative <grad u, n_tau>: its mean
    over every flat triangle (collapsed q x q Gauss rule)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    _, n = _areas_normals(verts, tris)
    U, W = triangle_rule(q)
    a, b, c = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    X = a[:, None, :] + U[None, :, :1] * (b - a)[:, None, :] + U[None, :, 1:2] * (c - b)[:, None, :]
    dn = np.einsum("ikd,id->ik", grad_u(X), n)
    return (dn * W[None, :]).sum(axis=1) / W.sum()


def energy_norm(G, e):
    """sqrt(e^T G e), the norm that the single-layer matrix G defines on
    piecewise constant coefficient vectors (an approximation of the
    H^{-1/2} norm of the function)."""
    e = np.asarray(e, dtype=np.float64)
    return math.sqrt(float(e @ (G @ e)))


def neumann_energy_error(G, verts, tris, t, grad_u, q=6):
    """||Pi t - t_h||_G: the discrete H^{-1/2} error of the Neumann
    coefficients t against the P0 projection of <grad u, n_tau>."""
    return energy_norm(G, neumann_projection(verts, tris, grad_u, q) - np.asarray(t, dtype=np.float64))
