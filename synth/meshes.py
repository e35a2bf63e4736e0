"""Seeded synthetic surface meshes and vectors.

All meshes are flat-triangle surface meshes given as ``(verts, tris)`` with
``verts`` float64 (nv, 3) and ``tris`` int32 (nt, 3); triangles are ordered
counter-clockwise seen from outside, so (b-a) x (c-a) points outward.
"""
import itertools
import math

import numpy as np


def random_vector(n, seed, cols=None):
    """x ~ N(0,1) from numpy's PCG64 generator; ``cols`` gives an (n, cols)
    column-major-compatible array (Fortran order)."""
    rng = np.random.default_rng(seed)
    if cols is None:
        return rng.standard_normal(n)
    return np.asfortranarray(rng.standard_normal((cols, n)).T)


def octa_sphere(s, project=True):
    """Sphere mesh of Section 5: the double pyramid |x1|+|x2|+|x3| = 1, each of
    its eight faces split regularly into s*s triangles, all vertices projected
    once to the unit sphere.  nt = 8 s^2, nv = 4 s^2 + 2.

    Vertex numbering: sorted by the integer lattice point (a, b, c) with
    |a|+|b|+|c| = s that the vertex comes from.  Triangle numbering: face by
    face (sign patterns in itertools.product((1,-1), repeat=3) order), then
    lattice rows."""
    if s < 1:
        raise ValueError("s must be >= 1")
    # local lattice of one face: points (i, j), i, j >= 0, i + j <= s, stored
    # row by row (j ascending, then i); row j starts at j (s+1) - j (j-1)/2
    jj = np.concatenate([np.full(s + 1 - j, j, dtype=np.int64) for j in range(s + 1)])
    ii = np.concatenate([np.arange(s + 1 - j, dtype=np.int64) for j in range(s + 1)])

    def lid(i, j):
        return j * (s + 1) - (j * (j - 1)) // 2 + i

    loc = []
    for j in range(s):
        i = np.arange(s - j, dtype=np.int64)
        up = np.stack([lid(i, j), lid(i + 1, j), lid(i, j + 1)], axis=1)
        i2 = i[i + j < s - 1]
        dn = np.stack([lid(i2 + 1, j), lid(i2 + 1, j + 1), lid(i2, j + 1)], axis=1)
        row = np.empty((len(up) + len(dn), 3), dtype=np.int64)
        row[0::2] = up
        row[1::2] = dn
        loc.append(row)
    loc = np.concatenate(loc)

    eye = np.eye(3, dtype=np.int64)
    keys_all, tris_all = [], []
    for f, (sx, sy, sz) in enumerate(itertools.product((1, -1), repeat=3)):
        A, B, C = sx * eye[0], sy * eye[1], sz * eye[2]
        if sx * sy * sz < 0:
            B, C = C, B
        pts = (s - ii - jj)[:, None] * A + ii[:, None] * B + jj[:, None] * C
        key = ((pts[:, 0] + s) * (2 * s + 1) + (pts[:, 1] + s)) * (2 * s + 1) + (pts[:, 2] + s)
        keys_all.append(key)
        tris_all.append(loc + f * len(ii))
    keys = np.concatenate(keys_all)
    uniq, inv = np.unique(keys, return_inverse=True)
    tris = inv[np.concatenate(tris_all)].astype(np.int32)
    a = uniq // ((2 * s + 1) ** 2) - s
    b = (uniq // (2 * s + 1)) % (2 * s + 1) - s
    c = uniq % (2 * s + 1) - s
    verts = np.stack([a, b, c], axis=1).astype(np.float64) / s
    if project:
        verts /= np.linalg.norm(verts, axis=1)[:, None]
    return verts, np.ascontiguousarray(tris)


def ellipsoid(s, a, b, c):
    """Octahedral unit sphere with every vertex scaled by (a, b, c) per axis."""
    v, t = octa_sphere(s)
    return v * np.array([a, b, c], dtype=np.float64)[None, :], t


def real_sph_harm(l, m, theta, phi):
    """Real orthonormal spherical harmonic Y_lm (no Condon-Shortley phase);
    theta = polar angle, phi = azimuth."""
    from scipy.special import lpmv
    am = abs(m)
    norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
    # scipy's lpmv carries the (-1)^m phase; remove it
    P = lpmv(am, l, np.cos(theta)) * (-1) ** am
    if m == 0:
        return norm * P
    if m > 0:
        return math.sqrt(2.0) * norm * P * np.cos(am * phi)
    return math.sqrt(2.0) * norm * P * np.sin(am * phi)


def perturbed_sphere(s, seed, lmax=8, amp=0.1):
    """Octahedral sphere with every projected vertex moved radially to
    r = 1 + amp * sum_{l<=lmax, |m|<=l} c_lm Y_lm, c_lm ~ N(0,1)/(l+1)^2 drawn
    in (l ascending, m ascending) order from ``seed``."""
    v, t = octa_sphere(s)
    rng = np.random.default_rng(seed)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    r = np.ones(len(v))
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            c = rng.standard_normal() / (l + 1) ** 2
            r += amp * c * real_sph_harm(l, m, theta, phi)
    return v * r[:, None], t


def flat_plate(n, size=1.0):
    """Planar square [0,size]^2 x {0} split into 2 n^2 triangles (normals +z)."""
    xs = np.linspace(0.0, size, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], axis=1)
    tris = []
    for j in range(n):
        for i in range(n):
            p = j * (n + 1) + i
            tris.append((p, p + 1, p + n + 2))
            tris.append((p, p + n + 2, p + n + 1))
    return verts, np.array(tris, dtype=np.int32)


def single_pair(kind, angle_deg=120.0):
    """Two triangles in a given relation: 'identical', 'edge' (common edge with
    the given dihedral opening angle), 'vertex', or 'disjoint'."""
    a = np.array([0.0, 0.0, 0.0])
    b = np.array([1.0, 0.0, 0.0])
    c = np.array([0.35, 0.8, 0.0])
    if kind == "identical":
        return np.array([a, b, c]), np.array([[0, 1, 2], [0, 1, 2]], dtype=np.int32)
    if kind == "edge":
        th = math.radians(angle_deg)
        d = np.array([0.55, 0.9 * math.cos(th), 0.9 * math.sin(th)])
        return np.array([a, b, c, d]), np.array([[0, 1, 2], [1, 0, 3]], dtype=np.int32)
    if kind == "vertex":
        d = np.array([-0.7, -0.35, 0.25])
        e = np.array([-0.2, -0.9, -0.3])
        return np.array([a, b, c, d, e]), np.array([[0, 1, 2], [0, 3, 4]], dtype=np.int32)
    if kind == "disjoint":
        d = np.array([0.2, 0.1, 0.5])
        return (np.array([a, b, c, a + d, b + d, c + d]),
                np.array([[0, 1, 2], [3, 5, 4]], dtype=np.int32))
    raise ValueError(kind)
