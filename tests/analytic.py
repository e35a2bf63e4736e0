"""Closed-form single-triangle potentials used to pin the quadrature oracle.

These are independent of the oracle's pair quadrature: the inner integral over
the source triangle is evaluated analytically, and only the outer integral is
done numerically (composite Gauss rule on a uniform 4^L subdivision).

* Single layer of a uniformly charged flat triangle, int_tau 1/|x-y| dy: the
  classical edge-sum formula (logarithms and arctangents per edge).
* Double layer of a flat triangle with unit density, int_tau <y-x,n>/|y-x|^3 dy:
  the signed solid angle of the triangle seen from x (Van Oosterom-Strackee).
"""
import math

import numpy as np


def slp_potential(tri, X):
    """int_tau 1/|x - y| dy for points X (n, 3); tri = (3, 3) corners."""
    r1, r2, r3 = tri
    n = np.cross(r2 - r1, r3 - r1)
    n = n / np.linalg.norm(n)
    d = (X - r1) @ n
    rho = X - d[:, None] * n[None, :]
    ad = np.abs(d)
    out = np.zeros(len(X))
    for ra, rb in ((r1, r2), (r2, r3), (r3, r1)):
        e = rb - ra
        le = e / np.linalg.norm(e)
        u = np.cross(le, n)
        lp = (rb - rho) @ le
        lm = (ra - rho) @ le
        t = (ra - rho) @ u
        R0sq = t * t + d * d
        Rp = np.linalg.norm(X - rb, axis=1)
        Rm = np.linalg.norm(X - ra, axis=1)
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.log((Rp + lp) / (Rm + lm))
            term = t * lg - ad * (np.arctan(t * lp / (R0sq + ad * Rp))
                                  - np.arctan(t * lm / (R0sq + ad * Rm)))
        term = np.where(np.abs(t) < 1e-14, 0.0, term)
        out += term
    return out


def solid_angle(tri, X):
    """Signed solid angle int_tau <y - x, n>/|y - x|^3 dy, n = unit normal of
    tri in its stored corner order."""
    a = tri[0][None, :] - X
    b = tri[1][None, :] - X
    c = tri[2][None, :] - X
    la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
           + np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
    return 2.0 * np.arctan2(num, den)


def subdivided_rule(tri, level, q):
    """Points and weights of a composite collapsed Gauss rule (q x q per
    sub-triangle) on a uniform 4^level subdivision of tri."""
    z, w = np.polynomial.legendre.leggauss(q)
    t = 0.5 * (z + 1.0)
    w = 0.5 * w
    U = np.array([(t[i], t[i] * t[j]) for i in range(q) for j in range(q)])
    W = np.array([w[i] * w[j] * t[i] for i in range(q) for j in range(q)])
    subs = [np.array(tri, dtype=np.float64)]
    for _ in range(level):
        nxt = []
        for s in subs:
            a, b, c = s
            ab, bc, ca = 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)
            nxt += [np.array([a, ab, ca]), np.array([ab, b, bc]),
                    np.array([ca, bc, c]), np.array([bc, ca, ab])]
        subs = nxt
    P, Wt = [], []
    for s in subs:
        P0, P1, P2 = s
        J = np.linalg.norm(np.cross(P1 - P0, P2 - P1))
        P.append(P0[None, :] + U[:, :1] * (P1 - P0)[None, :] + U[:, 1:2] * (P2 - P1)[None, :])
        Wt.append(W * J)
    return np.concatenate(P), np.concatenate(Wt)


def pair_slp_reference(tx, ty, level=5, q=6):
    """int_tx int_ty g(x,y) dy dx with the inner integral in closed form."""
    P, W = subdivided_rule(tx, level, q)
    return float(np.sum(W * slp_potential(ty, P))) / (4.0 * math.pi)


def pair_dlp_constant_reference(tx, ty, level=5, q=6):
    """int_tx int_ty dg/dn_y(x,y) dy dx (unit density) = -int_tx Omega(x)/(4 pi) dx."""
    P, W = subdivided_rule(tx, level, q)
    return -float(np.sum(W * solid_angle(ty, P))) / (4.0 * math.pi)
