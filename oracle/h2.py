"""Test infrastructure only: the interpolation-based H^2 approximation written
out as dense matrices (small meshes only).

Follows the paper's definitions directly, with no transfer matrices, no
blocking beyond the block tree, and no reordering:

* cluster tree (Section 2, Definition "Cluster tree"): recursive bisection of
  the bounding box of the clusters' characteristic points (triangle centroids
  for the piecewise-constant space, vertices for the piecewise-linear space) at
  the midpoint of its longest side, while a cluster holds more than ``leaf``
  indices;
* bounding boxes B_t containing the supports of all basis functions of t and
  the admissibility condition max(diam B_t, diam B_s) <= 2 eta dist(B_t, B_s)
  (Section 3, eq. (admissibility));
* block tree (Section 2, Definition "Block tree") with farfield leaves (the
  admissible blocks) and nearfield leaves (both clusters leaves);
* m-th order tensor Chebyshev interpolation of g on B_t x B_s (Section 3):
  G|_{t x s} ~ V_t S_ts W_s^T with (V_t)_{i nu} = int psi_i L_{t,nu},
  S_ts = (g(xi_{t,nu}, xi_{s,mu})), (W_s)_{j mu} = int psi_j L_{s,mu} for G and
  (W_s)_{j mu} = int phi_j dL_{s,mu}/dn for K (Section 5: derivatives of the
  approximated kernel).

Nearfield entries come from the dense quadrature oracle in ``bem_oracle.c``.
"""
import math

import numpy as np

from . import slp_dense, dlp_dense

FOUR_PI = 4.0 * math.pi


# ------------------------------------------------------------ cluster tree

class Cluster:
    __slots__ = ("idx", "children", "begin", "end", "lo", "hi", "level", "id")

    def __init__(self, idx, level):
        self.idx = idx
        self.children = []
        self.level = level


def cluster_tree(points, leaf):
    """Returns (root, perm, clusters).  ``perm[k]`` is the original index at
    position k of the cluster ordering; every cluster covers perm[begin:end].
    Clusters are listed in depth-first pre-order, first child first."""
    points = np.asarray(points, dtype=np.float64)
    clusters = []

    def split(idx, level):
        c = Cluster(idx, level)
        c.id = len(clusters)
        clusters.append(c)
        if len(idx) <= leaf:
            return c
        p = points[idx]
        lo = p.min(axis=0)
        hi = p.max(axis=0)
        ext = hi - lo
        axes = sorted(range(3), key=lambda a: (-ext[a], a))
        for ax in axes:
            mid = 0.5 * (lo[ax] + hi[ax])
            first = p[:, ax] <= mid
            if first.all() or not first.any():
                continue
            c.children = [split(idx[first], level + 1), split(idx[~first], level + 1)]
            break
        return c

    root = split(np.arange(len(points)), 0)
    perm = []

    def order(c):
        c.begin = len(perm)
        if not c.children:
            perm.extend(c.idx.tolist())
        for ch in c.children:
            order(ch)
        c.end = len(perm)

    order(root)
    return root, np.array(perm, dtype=np.int64), clusters


def support_boxes(clusters, verts, tris, space):
    """Axis-parallel boxes containing the supports of the basis functions:
    space 'P0' -> triangles (support = the triangle), 'P1' -> vertices
    (support = all triangles around the vertex)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris)
    if space == "P1":
        adj = [[] for _ in range(len(verts))]
        for k, t in enumerate(tris):
            for v in t:
                adj[v].append(k)
    for c in clusters:
        if space == "P0":
            vs = tris[c.idx].ravel()
        else:
            ts = sorted({k for v in c.idx for k in adj[v]})
            vs = tris[ts].ravel()
        c.lo = verts[vs].min(axis=0)
        c.hi = verts[vs].max(axis=0)


def diam(c):
    return math.sqrt(float(np.sum((c.hi - c.lo) ** 2)))


def dist(t, s):
    gap = np.maximum(0.0, np.maximum(s.lo - t.hi, t.lo - s.hi))
    return math.sqrt(float(np.sum(gap ** 2)))


def admissible(t, s, eta):
    return max(diam(t), diam(s)) <= 2.0 * eta * dist(t, s)


def block_tree(rt, cs, eta, disable_far=False):
    """Farfield leaves (admissible) and nearfield leaves (both leaves)."""
    far, near = [], []

    def rec(t, s):
        if not disable_far and admissible(t, s, eta):
            far.append((t, s))
        elif not t.children and not s.children:
            near.append((t, s))
        elif not t.children:
            for s2 in s.children:
                rec(t, s2)
        elif not s.children:
            for t2 in t.children:
                rec(t2, s)
        else:
            for t2 in t.children:
                for s2 in s.children:
                    rec(t2, s2)

    rec(rt, cs)
    return far, near


# --------------------------------------------------- Chebyshev interpolation

def cheb_points_1d(a, b, m):
    """First-kind Chebyshev points on [a, b]: (a+b)/2 + (b-a)/2 cos(pi (2i+1)/(2m))."""
    i = np.arange(m)
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos(math.pi * (2 * i + 1) / (2 * m))


def box_axes(c, m):
    """Per-axis interpolation points of the box of cluster c (degenerate sides
    widened to 1e-12 diam)."""
    d = diam(c)
    axes = []
    for k in range(3):
        a, b = float(c.lo[k]), float(c.hi[k])
        if b - a < 1e-12 * d:
            mid = 0.5 * (a + b)
            a, b = mid - 0.5e-12 * d, mid + 0.5e-12 * d
        axes.append(cheb_points_1d(a, b, m))
    return axes


def tensor_points(axes):
    """xi_nu with nu = nu1 + m nu2 + m^2 nu3."""
    m = len(axes[0])
    P = np.zeros((m ** 3, 3))
    for n3 in range(m):
        for n2 in range(m):
            for n1 in range(m):
                P[n1 + m * n2 + m * m * n3] = (axes[0][n1], axes[1][n2], axes[2][n3])
    return P


def lagrange_1d(pts, z):
    """ell_i(z) for all i, z array -> (len(z), m)."""
    z = np.asarray(z, dtype=np.float64)
    m = len(pts)
    out = np.ones((len(z), m))
    for i in range(m):
        for j in range(m):
            if j != i:
                out[:, i] *= (z - pts[j]) / (pts[i] - pts[j])
    return out


def lagrange_1d_deriv(pts, z):
    """d ell_i / dz (product rule)."""
    z = np.asarray(z, dtype=np.float64)
    m = len(pts)
    out = np.zeros((len(z), m))
    for i in range(m):
        for k in range(m):
            if k == i:
                continue
            term = np.full(len(z), 1.0 / (pts[i] - pts[k]))
            for j in range(m):
                if j != i and j != k:
                    term = term * (z - pts[j]) / (pts[i] - pts[j])
            out[:, i] += term
    return out


def lagrange_tensor(axes, X):
    """L_nu(x) for points X (n, 3) -> (n, m^3)."""
    m = len(axes[0])
    l = [lagrange_1d(axes[d], X[:, d]) for d in range(3)]
    out = np.zeros((len(X), m ** 3))
    for n3 in range(m):
        for n2 in range(m):
            for n1 in range(m):
                out[:, n1 + m * n2 + m * m * n3] = l[0][:, n1] * l[1][:, n2] * l[2][:, n3]
    return out


def lagrange_tensor_grad(axes, X):
    """grad L_nu(x) -> (n, m^3, 3)."""
    m = len(axes[0])
    l = [lagrange_1d(axes[d], X[:, d]) for d in range(3)]
    dl = [lagrange_1d_deriv(axes[d], X[:, d]) for d in range(3)]
    out = np.zeros((len(X), m ** 3, 3))
    for n3 in range(m):
        for n2 in range(m):
            for n1 in range(m):
                nu = n1 + m * n2 + m * m * n3
                out[:, nu, 0] = dl[0][:, n1] * l[1][:, n2] * l[2][:, n3]
                out[:, nu, 1] = l[0][:, n1] * dl[1][:, n2] * l[2][:, n3]
                out[:, nu, 2] = l[0][:, n1] * l[1][:, n2] * dl[2][:, n3]
    return out


# ------------------------------------------------------ triangle quadrature

def triangle_rule(q):
    """Collapsed Gauss rule on the reference triangle {0 <= u2 <= u1 <= 1}:
    points (a, a b), weights w_a w_b a (numpy's Gauss-Legendre)."""
    z, w = np.polynomial.legendre.leggauss(q)
    t = 0.5 * (z + 1.0)
    w = 0.5 * w
    U = np.array([(t[a], t[a] * t[b]) for a in range(q) for b in range(q)])
    W = np.array([w[a] * w[b] * t[a] for a in range(q) for b in range(q)])
    return U, W


def _tri_points(verts, tri, U):
    P0, P1, P2 = verts[tri[0]], verts[tri[1]], verts[tri[2]]
    X = P0[None, :] + U[:, :1] * (P1 - P0)[None, :] + U[:, 1:2] * (P2 - P1)[None, :]
    J = np.linalg.norm(np.cross(P1 - P0, P2 - P1))
    return X, J


def basis_p0(verts, tris, idx, axes, q):
    """(V_t)_{i nu} = int_{tau_i} L_{t,nu}(x) dx."""
    U, W = triangle_rule(q)
    V = np.zeros((len(idx), len(axes[0]) ** 3))
    for r, i in enumerate(idx):
        X, J = _tri_points(verts, tris[i], U)
        V[r] = J * (W[:, None] * lagrange_tensor(axes, X)).sum(axis=0)
    return V


def basis_p1_normal_derivative(verts, tris, adj, idx, axes, q):
    """(W_s)_{j mu} = sum_{tau around j} int_tau phi_j(y) <grad L_{s,mu}(y), n_tau> dy."""
    U, W = triangle_rule(q)
    out = np.zeros((len(idx), len(axes[0]) ** 3))
    for r, j in enumerate(idx):
        for k in adj[j]:
            tri = tris[k]
            X, J = _tri_points(verts, tri, U)
            a, b, c = verts[tri[0]], verts[tri[1]], verts[tri[2]]
            n = np.cross(b - a, c - a)
            n /= np.linalg.norm(n)
            lam = np.stack([1.0 - U[:, 0], U[:, 0] - U[:, 1], U[:, 1]], axis=1)
            slot = list(tri).index(j)
            dn = lagrange_tensor_grad(axes, X) @ n
            out[r] += J * ((W * lam[:, slot])[:, None] * dn).sum(axis=0)
    return out


def coupling(axes_t, axes_s):
    """S_ts[nu, mu] = g(xi_{t,nu}, xi_{s,mu})."""
    Pt = tensor_points(axes_t)
    Ps = tensor_points(axes_s)
    d = np.linalg.norm(Pt[:, None, :] - Ps[None, :, :], axis=2)
    return 1.0 / (FOUR_PI * d)


# ----------------------------------------------------------- dense H^2

def h2_dense(verts, tris, kernel, leaf, m, eta=1.0, q_near=4, q_basis=None,
             near_matrix=None, disable_far=False):
    """Dense matrix of the interpolation-based H^2 approximation of G
    (kernel 'slp') or K (kernel 'dlp').  Returns (A, info)."""
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    if q_basis is None:
        q_basis = 2 * m + 1
    cent = verts[tris].mean(axis=1)
    rt, rperm, rcl = cluster_tree(cent, leaf)
    support_boxes(rcl, verts, tris, "P0")
    if kernel == "slp":
        ct, cperm, ccl = rt, rperm, rcl
        ncols = len(tris)
        dense = slp_dense if near_matrix is None else None
    else:
        ct, cperm, ccl = cluster_tree(verts, leaf)
        support_boxes(ccl, verts, tris, "P1")
        ncols = len(verts)
        dense = dlp_dense if near_matrix is None else None
    full = near_matrix if near_matrix is not None else dense(verts, tris, q_near)
    far, near = block_tree(rt, ct, eta, disable_far=disable_far)
    A = np.zeros((len(tris), ncols))
    for (t, s) in near:
        ri = rperm[t.begin:t.end]
        ci = cperm[s.begin:s.end]
        A[np.ix_(ri, ci)] = full[np.ix_(ri, ci)]
    adj = None
    if kernel == "dlp":
        adj = [[] for _ in range(len(verts))]
        for k, t in enumerate(tris):
            for v in t:
                adj[v].append(k)
    cacheV, cacheW = {}, {}
    for (t, s) in far:
        if t.id not in cacheV:
            cacheV[t.id] = basis_p0(verts, tris, rperm[t.begin:t.end], box_axes(t, m), q_basis)
        if s.id not in cacheW:
            ax = box_axes(s, m)
            if kernel == "slp":
                cacheW[s.id] = basis_p0(verts, tris, cperm[s.begin:s.end], ax, q_basis)
            else:
                cacheW[s.id] = basis_p1_normal_derivative(verts, tris, adj, cperm[s.begin:s.end],
                                                          ax, q_basis)
        S = coupling(box_axes(t, m), box_axes(s, m))
        ri = rperm[t.begin:t.end]
        ci = cperm[s.begin:s.end]
        A[np.ix_(ri, ci)] = cacheV[t.id] @ S @ cacheW[s.id].T
    info = dict(far=len(far), near=len(near), row_clusters=len(rcl), col_clusters=len(ccl),
                row_perm=rperm, col_perm=cperm, row_tree=rcl, col_tree=ccl,
                far_blocks=[(t.id, s.id) for t, s in far],
                near_blocks=[(t.id, s.id) for t, s in near])
    return A, info


# ------------------------------------------- sampled rows of the H^2 matrix
#
# For meshes whose dense H^2 matrix is too large to write out, the rows of
# A X for a few row indices: the same trees, block tree, interpolation bases,
# couplings and near-field entries as h2_dense, summed block by block for
# each requested row without forming A.

def _tensor_quad(wq, a, b, c):
    """Quadrature of tensor products: out[n, nu] = sum_q wq[n, q] a[n, q, n1]
    b[n, q, n2] c[n, q, n3] with nu = n1 + m n2 + m^2 n3 (one batched matrix
    product over q per row n)."""
    n, Q, m = a.shape
    B = wq[:, :, None, None] * c[:, :, :, None] * b[:, :, None, :]
    return np.matmul(B.reshape(n, Q, m * m).transpose(0, 2, 1), a).reshape(n, m ** 3)


def _factors(axes, X, f):
    """f(axes[d], X[..., d]) per axis, shaped like X[..., 0] plus one axis."""
    return [f(axes[d], X[..., d].ravel()).reshape(X.shape[:-1] + (len(axes[d]),)) for d in range(3)]


def basis_p0_many(verts, tris, idx, axes, q, chunk=2048):
    """(V_t)_{i nu} = int_{tau_i} L_{t,nu} for many triangles at once (the
    same collapsed rule as basis_p0)."""
    U, W = triangle_rule(q)
    idx = np.asarray(idx, dtype=np.int64)
    out = np.zeros((len(idx), len(axes[0]) ** 3))
    for c0 in range(0, len(idx), chunk):
        tr = tris[idx[c0:c0 + chunk]]
        P0, P1, P2 = verts[tr[:, 0]], verts[tr[:, 1]], verts[tr[:, 2]]
        X = P0[:, None, :] + U[None, :, :1] * (P1 - P0)[:, None, :] + U[None, :, 1:2] * (P2 - P1)[:, None, :]
        J = np.linalg.norm(np.cross(P1 - P0, P2 - P1), axis=1)
        l = _factors(axes, X, lagrange_1d)
        out[c0:c0 + len(tr)] = J[:, None] * _tensor_quad(np.broadcast_to(W, (len(tr), len(W))), *l)
    return out


def basis_p1_nd_many(verts, tris, adj, idx, axes, q):
    """(W_s)_{j mu} = sum_{tau around j} int_tau phi_j <grad L_{s,mu}, n_tau>
    for many vertices at once (the same rule as basis_p1_normal_derivative)."""
    inc_row, inc_tri, inc_slot = [], [], []
    for r, j in enumerate(idx):
        for k in adj[j]:
            inc_row.append(r)
            inc_tri.append(k)
            inc_slot.append(list(tris[k]).index(j))
    return _basis_p1_nd_incidences(verts, tris, len(idx), np.asarray(inc_row, dtype=np.int64),
                                   np.asarray(inc_tri, dtype=np.int64), np.asarray(inc_slot, dtype=np.int64),
                                   axes, q)


def _basis_p1_nd_incidences(verts, tris, nrows, inc_row, inc_tri, inc_slot, axes, q, chunk=1024):
    """Sum over incidences (row r, triangle tau, corner slot c of the row's
    vertex in tau) of int_tau lambda_c <grad L_mu, n_tau> into row r."""
    U, W = triangle_rule(q)
    lam = np.stack([1.0 - U[:, 0], U[:, 0] - U[:, 1], U[:, 1]], axis=1)
    m = len(axes[0])
    out = np.zeros((nrows, m ** 3))
    for c0 in range(0, len(inc_row), chunk):
        tr = tris[inc_tri[c0:c0 + chunk]]
        P0, P1, P2 = verts[tr[:, 0]], verts[tr[:, 1]], verts[tr[:, 2]]
        X = P0[:, None, :] + U[None, :, :1] * (P1 - P0)[:, None, :] + U[None, :, 1:2] * (P2 - P1)[:, None, :]
        J = np.linalg.norm(np.cross(P1 - P0, P2 - P1), axis=1)
        nrm = np.cross(P1 - P0, P2 - P0)
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        l = _factors(axes, X, lagrange_1d)
        dl = _factors(axes, X, lagrange_1d_deriv)
        wl = W[None, :] * lam[:, inc_slot[c0:c0 + chunk]].T
        dn = (_tensor_quad(wl * nrm[:, :1], dl[0], l[1], l[2]) + _tensor_quad(wl * nrm[:, 1:2], l[0], dl[1], l[2])
              + _tensor_quad(wl * nrm[:, 2:3], l[0], l[1], dl[2]))
        np.add.at(out, inc_row[c0:c0 + chunk], J[:, None] * dn)
    return out


def h2_rows(verts, tris, kernel, leaf, m, rows, X, eta=1.0, q_near=4, q_basis=None):
    """Rows ``rows`` of A X for the H^2 matrix A that h2_dense writes out
    (kernel 'slp' or 'dlp'); X has one row per column of A (vector or
    matrix).  Row i gets, from each nearfield leaf (t_i, s) of its leaf
    cluster t_i, the dense entries times X|_s, and from each farfield block
    (t, s) whose row cluster t contains i, V_t[i] S_ts (W_s^T X|_s)."""
    from . import slp_block, dlp_block
    verts = np.asarray(verts, dtype=np.float64)
    tris = np.asarray(tris, dtype=np.int64)
    X = np.asarray(X, dtype=np.float64)
    vec = X.ndim == 1
    X2 = X[:, None] if vec else X
    if q_basis is None:
        q_basis = 2 * m + 1
    cent = verts[tris].mean(axis=1)
    rt, rperm, rcl = cluster_tree(cent, leaf)
    support_boxes(rcl, verts, tris, "P0")
    if kernel == "slp":
        ct, cperm, ccl = rt, rperm, rcl
    else:
        ct, cperm, ccl = cluster_tree(verts, leaf)
        support_boxes(ccl, verts, tris, "P1")
    far, near = block_tree(rt, ct, eta)
    far_by_t, near_by_t = {}, {}
    for t, s in far:
        far_by_t.setdefault(t.id, []).append(s)
    for t, s in near:
        near_by_t.setdefault(t.id, []).append(s)
    if kernel == "dlp":
        # corner incidences (triangle, slot) sorted by their vertex's position
        # in the column cluster order: each vertex cluster owns one range
        cpos = np.empty(len(cperm), dtype=np.int64)
        cpos[cperm] = np.arange(len(cperm))
        key = cpos[tris.ravel()]
        order = np.argsort(key, kind="stable")
        inc_pos, inc_tri, inc_slot = key[order], order // 3, order % 3
    pos = np.empty(len(rperm), dtype=np.int64)
    pos[rperm] = np.arange(len(rperm))
    xhat = {}
    out = np.zeros((len(rows), X2.shape[1]))
    for r, i in enumerate(rows):
        p = pos[i]
        c = rt
        path = [c]
        while c.children:
            c = next(ch for ch in c.children if ch.begin <= p < ch.end)
            path.append(c)
        for t in path:
            if t.id not in far_by_t:
                continue
            ax_t = box_axes(t, m)
            Vi = basis_p0_many(verts, tris, [i], ax_t, q_basis)[0]
            for s in far_by_t[t.id]:
                if s.id not in xhat:
                    ax_s = box_axes(s, m)
                    cols = cperm[s.begin:s.end]
                    if kernel == "slp":
                        Ws = basis_p0_many(verts, tris, cols, ax_s, q_basis)
                    else:
                        a, b = np.searchsorted(inc_pos, [s.begin, s.end])
                        Ws = _basis_p1_nd_incidences(verts, tris, s.end - s.begin, inc_pos[a:b] - s.begin,
                                                     inc_tri[a:b], inc_slot[a:b], ax_s, q_basis)
                    xhat[s.id] = Ws.T @ X2[cols]
                out[r] += Vi @ coupling(ax_t, box_axes(s, m)) @ xhat[s.id]
        leaf_t = path[-1]
        cols = np.concatenate([cperm[s.begin:s.end] for s in near_by_t.get(leaf_t.id, [])] or
                              [np.zeros(0, dtype=np.int64)])
        if len(cols):
            ent = (slp_block if kernel == "slp" else dlp_block)(verts, tris, q_near, [i], cols)
            out[r] += ent[0] @ X2[cols]
    return out[:, 0] if vec else out
