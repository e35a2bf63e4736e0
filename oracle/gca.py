"""Test infrastructure only: the Green cross approximation (GCA) of the
single-layer matrix G (Section 4), written out as a dense matrix for small
meshes.

Steps, in the order of Section 4:

* For a cluster t with bounding box B_t = [a, b] take the auxiliary box
  omega_t = [a - delta_t, b + delta_t] with delta_t the largest side of B_t,
  so that dist(boundary of omega_t, B_t) = delta_t (Section 5).
* Green's representation formula on omega_t, for x in omega_t and y outside:
  g(x, y) = int g(x, z) dg/dn_z(z, y) dz - int dg/dn_z(x, z) g(z, y) dz over
  the boundary of omega_t, discretised by a quadrature rule (w_nu, z_nu):
  here an m x m Gauss-Legendre rule on each of the six faces.
* L = [A C] with a_{i nu} = w_nu^{1/2} int psi_i(x) g(x, z_nu) dx and
  c_{i nu} = w_nu^{1/2} int psi_i(x) dg/dn_z(x, z_nu) dx.
* Adaptive cross approximation of L: row pivots tau and column pivots sigma
  with L ~ L|_{t x sigma} (L|_{tau x sigma})^{-1} L|_{tau x [1:2k]}; here
  with full pivoting (the entry of largest modulus of the remainder) and
  stopped once that entry is at most eps times the first pivot.
* V_t = L|_{t x sigma} (L|_{tau x sigma})^{-1} and t_hat = tau, so that
  G|_{t x s} ~ V_t G|_{t_hat x s}.  Nested version: for a cluster with
  children the rows are t_hat_1 followed by t_hat_2 instead of t, L is built
  for those rows with the parent's omega_t, and [E_1; E_2] = V_hat_t.
* G|_{t x s} ~ V_t G|_{t_hat x s_hat} V_s^T for the farfield blocks (the same
  construction on the column cluster; for G both trees are the same), the
  entries G|_{t_hat x s_hat} taken from the dense Galerkin matrix.
* The double-layer matrix K "takes the appropriate derivatives" (Section 5):
  its rows use the same V_t (x -> dg/dn_y(x, y) is harmonic in omega_t too);
  its columns (hat functions phi_j on the vertices of a cluster s) apply
  Green's formula in y on omega_s and differentiate it in n_y, so that
  L_s = [B D] with b_{j nu} = w^{1/2} int phi_j(y) dg/dn_y(y, z_nu) dy and
  d_{j nu} = w^{1/2} int phi_j(y) d^2 g/(dn_y dn_z)(y, z_nu) dy, and
  K|_{t x s} ~ V_t K|_{t_hat x s_hat} W_s^T.

The triangle integrals of L use the collapsed Gauss rule with m + 2 points
per direction.
"""
import math

import numpy as np

from .h2 import block_tree, cluster_tree, support_boxes, triangle_rule

FOUR_PI = 4.0 * math.pi


def omega_box(lo, hi):
    """omega_t for the bounding box [lo, hi]: every side moved out by delta_t."""
    delta = float(np.max(hi - lo))
    return lo - delta, hi + delta


def face_rule(lo, hi, m):
    """m x m Gauss-Legendre points on each of the six faces of the box
    [lo, hi]: points z (6 m^2 x 3), weights w (face area included) and outward
    unit normals."""
    zq, wq = np.polynomial.legendre.leggauss(m)
    t, w1 = 0.5 * (zq + 1.0), 0.5 * wq
    Z, W, N = [], [], []
    for ax in range(3):
        o1, o2 = [a for a in range(3) if a != ax]
        for side, sgn in ((lo[ax], -1.0), (hi[ax], 1.0)):
            for i in range(m):
                for j in range(m):
                    z = np.zeros(3)
                    z[ax] = side
                    z[o1] = lo[o1] + t[i] * (hi[o1] - lo[o1])
                    z[o2] = lo[o2] + t[j] * (hi[o2] - lo[o2])
                    n = np.zeros(3)
                    n[ax] = sgn
                    Z.append(z)
                    W.append(w1[i] * w1[j] * (hi[o1] - lo[o1]) * (hi[o2] - lo[o2]))
                    N.append(n)
    return np.array(Z), np.array(W), np.array(N)


def green_matrix(verts, tris, rows, Z, W, N, q):
    """L = [A C] for the triangles `rows` (original indices)."""
    U, Wt = triangle_rule(q)
    k = len(Z)
    L = np.zeros((len(rows), 2 * k))
    sw = np.sqrt(W)
    for r, i in enumerate(rows):
        P0, P1, P2 = verts[tris[i, 0]], verts[tris[i, 1]], verts[tris[i, 2]]
        X = P0[None, :] + U[:, :1] * (P1 - P0)[None, :] + U[:, 1:2] * (P2 - P1)[None, :]
        jac = np.linalg.norm(np.cross(P1 - P0, P2 - P1))
        D = X[:, None, :] - Z[None, :, :]            # x - z
        R = np.linalg.norm(D, axis=2)
        g = 1.0 / (FOUR_PI * R)
        dg = np.einsum("qkd,kd->qk", D, N) / (FOUR_PI * R ** 3)   # n_z . grad_z g(x, z)
        L[r, :k] = sw * (Wt @ g) * jac
        L[r, k:] = sw * (Wt @ dg) * jac
    return L


def green_matrix_p1(verts, tris, adj, rows, Z, W, N, q):
    """L_s = [B D] for the vertices `rows` (hat functions, normal derivatives
    in y of Green's formula on the column box)."""
    U, Wt = triangle_rule(q)
    lam = np.stack([1.0 - U[:, 0], U[:, 0] - U[:, 1], U[:, 1]], axis=1)
    k = len(Z)
    L = np.zeros((len(rows), 2 * k))
    sw = np.sqrt(W)
    for r, j in enumerate(rows):
        for tri_id in adj[j]:
            tri = tris[tri_id]
            corner = int(np.where(tri == j)[0][0])
            P0, P1, P2 = verts[tri[0]], verts[tri[1]], verts[tri[2]]
            X = P0[None, :] + U[:, :1] * (P1 - P0)[None, :] + U[:, 1:2] * (P2 - P1)[None, :]
            cr = np.cross(P1 - P0, P2 - P1)
            jac = np.linalg.norm(cr)
            ny = cr / jac
            D = X[:, None, :] - Z[None, :, :]            # y - z
            R = np.linalg.norm(D, axis=2)
            dny = D @ ny                                  # n_y . (y - z)
            dnz = np.einsum("qkd,kd->qk", D, N)           # n_z . (y - z)
            b = -dny / (FOUR_PI * R ** 3)                 # dg/dn_y(y, z)
            d = (N @ ny)[None, :] / (FOUR_PI * R ** 3) - 3.0 * dny * dnz / (FOUR_PI * R ** 5)
            wl = Wt * lam[:, corner] * jac
            L[r, :k] += sw * (wl @ b)
            L[r, k:] += sw * (wl @ d)
    return L


def aca_full(L, eps):
    """Cross approximation with full pivoting: returns the row and column
    pivot lists (positions in L) in the order chosen."""
    R = np.array(L, dtype=np.float64)
    tau, sigma = [], []
    first = None
    for _ in range(min(R.shape)):
        flat = int(np.argmax(np.abs(R)))
        i, j = divmod(flat, R.shape[1])
        piv = R[i, j]
        if first is None:
            first = abs(piv)
            if first == 0.0:
                break
        elif abs(piv) <= eps * first:
            break
        tau.append(i)
        sigma.append(j)
        R = R - np.outer(R[:, j], R[i, :]) / piv
    return tau, sigma


def gca_bases(verts, tris, clusters, perm, m, eps, q=None, space="P0"):
    """Bottom-up GCA: for every cluster the pivot indices t_hat (original
    triangle indices, or vertex indices for space 'P1') and, for leaves, V_t
    (|t| x k_t in the cluster's position order) or, for parents, V_hat_t
    ((k_1 + k_2) x k_t)."""
    q = m + 2 if q is None else q
    hat, V = {}, {}
    adj = None
    if space == "P1":
        adj = [[] for _ in range(len(verts))]
        for k, tri in enumerate(tris):
            for v in tri:
                adj[v].append(k)
    for c in sorted(clusters, key=lambda c: -c.level):
        if c.children:
            rows = np.concatenate([hat[ch.id] for ch in c.children]).astype(np.int64)
        else:
            rows = perm[c.begin:c.end]
        lo, hi = omega_box(c.lo, c.hi)
        Z, W, N = face_rule(lo, hi, m)
        if space == "P1":
            L = green_matrix_p1(verts, tris, adj, rows, Z, W, N, q)
        else:
            L = green_matrix(verts, tris, rows, Z, W, N, q)
        tau, sigma = aca_full(L, eps)
        Ls = L[:, sigma]
        V[c.id] = np.linalg.solve(L[np.ix_(tau, sigma)].T, Ls.T).T
        hat[c.id] = rows[tau]
    return hat, V


def full_basis(c, V):
    """V_t on all |t| rows (position order) from the nested representation."""
    if not c.children:
        return V[c.id]
    blocks = [full_basis(ch, V) for ch in c.children]
    n = sum(b.shape[0] for b in blocks)
    k = sum(b.shape[1] for b in blocks)
    D = np.zeros((n, k))
    r = cc = 0
    for b in blocks:
        D[r:r + b.shape[0], cc:cc + b.shape[1]] = b
        r += b.shape[0]
        cc += b.shape[1]
    return D @ V[c.id]


def gca_dense(verts, tris, leaf, m, eps, G, eta=1.0):
    """Dense matrix of the GCA H^2 approximation of G (nearfield and the
    pivot entries taken from the dense Galerkin matrix G).  Returns (A, info)
    with the ranks and pivots."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    cent = verts[tris].mean(axis=1)
    root, perm, clusters = cluster_tree(cent, leaf)
    support_boxes(clusters, verts, tris, "P0")
    far, near = block_tree(root, root, eta)
    hat, V = gca_bases(verts, tris, clusters, perm, m, eps)
    A = np.zeros((len(tris), len(tris)))
    for t, s in near:
        ri, ci = perm[t.begin:t.end], perm[s.begin:s.end]
        A[np.ix_(ri, ci)] = G[np.ix_(ri, ci)]
    full = {}
    for t, s in far:
        for c in (t, s):
            if c.id not in full:
                full[c.id] = full_basis(c, V)
        ri, ci = perm[t.begin:t.end], perm[s.begin:s.end]
        A[np.ix_(ri, ci)] = full[t.id] @ G[np.ix_(hat[t.id], hat[s.id])] @ full[s.id].T
    info = dict(ranks={c.id: len(hat[c.id]) for c in clusters}, hat=hat, far=len(far), near=len(near))
    return A, info


def gca_dense_dlp(verts, tris, leaf, m, eps, K, eta=1.0):
    """Dense matrix of the GCA H^2 approximation of K (triangle rows,
    vertex columns; nearfield and pivot entries from the dense K)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    cent = verts[tris].mean(axis=1)
    rt, rperm, rcl = cluster_tree(cent, leaf)
    support_boxes(rcl, verts, tris, "P0")
    ct, cperm, ccl = cluster_tree(verts, leaf)
    support_boxes(ccl, verts, tris, "P1")
    far, near = block_tree(rt, ct, eta)
    rhat, RV = gca_bases(verts, tris, rcl, rperm, m, eps)
    chat, CV = gca_bases(verts, tris, ccl, cperm, m, eps, space="P1")
    A = np.zeros((len(tris), len(verts)))
    for t, s in near:
        ri, ci = rperm[t.begin:t.end], cperm[s.begin:s.end]
        A[np.ix_(ri, ci)] = K[np.ix_(ri, ci)]
    rf, cf = {}, {}
    for t, s in far:
        if t.id not in rf:
            rf[t.id] = full_basis(t, RV)
        if s.id not in cf:
            cf[s.id] = full_basis(s, CV)
        ri, ci = rperm[t.begin:t.end], cperm[s.begin:s.end]
        A[np.ix_(ri, ci)] = rf[t.id] @ K[np.ix_(rhat[t.id], chat[s.id])] @ cf[s.id].T
    info = dict(row_ranks={c.id: len(rhat[c.id]) for c in rcl}, col_ranks={c.id: len(chat[c.id]) for c in ccl},
                far=len(far), near=len(near))
    return A, info
