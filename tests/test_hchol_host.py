"""The H-Cholesky preconditioner on the host (no GPU): the oracle's dense-
storage factorisation pinned to the Cholesky factorisation and to its
accuracy bound, and the library's H-matrix factorisation (coarsening,
truncated low-rank arithmetic) against both, on the single-layer matrix of
small spheres."""
import numpy as np
import pytest

import oracle
import synth
from oracle import h2, hchol, krylov


def _lib():
    import paper_2001_05523_amd as h
    return h


def _setup(s, leaf, seed=None):
    v, t = synth.octa_sphere(s) if seed is None else synth.perturbed_sphere(s, seed)
    G = oracle.slp_dense(v, t, 4)
    root, perm, cl = h2.cluster_tree(v[t].mean(axis=1), leaf)
    h2.support_boxes(cl, v, t, "P0")
    far, _ = h2.block_tree(root, root, 1.0)
    return v, t, G, root, perm, far


# ---------------------------------------------------------- oracle pins

@pytest.mark.parametrize("s,leaf", [(4, 8), (8, 16)])
def test_oracle_without_truncation_is_the_cholesky_factor(s, leaf):
    """eps = 0: nothing is truncated and the recursion is the block form of
    the Cholesky factorisation, so L equals numpy's factor."""
    _, _, G, root, perm, far = _setup(s, leaf)
    Gp = G[np.ix_(perm, perm)]
    L = hchol.hchol(Gp, root, far, 0.0)
    Lref = np.linalg.cholesky(Gp)
    assert np.max(np.abs(L - Lref)) <= 1e-12 * np.max(np.abs(Lref))


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6])
def test_oracle_factor_reaches_its_accuracy(eps):
    """eps > 0: L L^T reproduces A to about eps (blockwise truncations of
    relative size eps, a few per block), L is lower triangular with a
    positive diagonal, and truncation actually happened (the low-rank blocks
    of L have rank below their size)."""
    _, _, G, root, perm, far = _setup(8, 16)
    Gp = G[np.ix_(perm, perm)]
    L = hchol.hchol(Gp, root, far, eps)
    assert np.array_equal(L, np.tril(L)) and np.all(np.diag(L) > 0)
    err = np.linalg.norm(L @ L.T - Gp, 2) / np.linalg.norm(Gp, 2)
    assert eps / 1e3 < err <= 10 * eps, err
    low = hchol.lowrank_blocks(Gp, root, far, eps)
    assert low
    ranks = [np.linalg.matrix_rank(L[t.begin:t.end, s.begin:s.end], tol=1e-14 * np.abs(L).max())
             for t, s in low]
    assert max(ranks) < max(min(t.end - t.begin, s.end - s.begin) for t, s in low)


def test_oracle_truncation_definition():
    """truncate() keeps exactly the singular values above eps * the largest."""
    rng = np.random.default_rng(7)
    U, _ = np.linalg.qr(rng.standard_normal((12, 6)))
    V, _ = np.linalg.qr(rng.standard_normal((9, 6)))
    sig = np.array([1.0, 0.5, 1e-2, 1e-3, 1e-5, 1e-9])
    B = (U * sig) @ V.T
    for eps, k in [(0.6, 1), (2e-3, 3), (1e-6, 5), (0.0, 6)]:
        T = hchol.truncate(B, eps)
        assert np.linalg.matrix_rank(T, tol=1e-12) == k
        assert np.linalg.norm(T - (U[:, :k] * sig[:k]) @ V[:, :k].T) <= 1e-14


def test_oracle_preconditioner_reduces_iterations():
    _, _, G, root, perm, far = _setup(8, 16)
    Gp = G[np.ix_(perm, perm)]
    b = synth.random_vector(len(Gp), 11)
    L = hchol.hchol(Gp, root, far, 1e-2)
    _, it_pc, _ = krylov.pcg(lambda p: Gp @ p, lambda r: hchol.solve(L, r), b, 1e-10, 500)
    _, it_cg, _ = krylov.cg(lambda p: Gp @ p, b, 1e-10, 500)
    assert it_pc <= 10 < it_cg


# ------------------------------------------------- library against oracle

@pytest.mark.parametrize("s,leaf,seed", [(4, 8, None), (8, 16, None), (8, 8, 31)])
def test_library_exact_factor_equals_cholesky_solve(s, leaf, seed):
    """eps = 0: the library's H-matrix factorisation solves G z = b like the
    dense Cholesky factor (numpy) and like the oracle's factor.  Both read
    only the lower triangle, and the quadrature makes G symmetric only up to
    its error for touching pairs, so the reference is the symmetric matrix
    with G's lower triangle."""
    h = _lib()
    v, t, G, root, perm, far = _setup(s, leaf, seed)
    m = h.Mesh(v, t)
    T = h.Tree(m, 0, leaf)
    P = h.HChol.from_dense(h.Blocks(T, T, 1.0), G, 0.0)
    b = synth.random_vector(len(t), 12)
    z = P.solve_host(b)
    Gp = G[np.ix_(perm, perm)]
    Gl = np.tril(Gp) + np.tril(Gp, -1).T
    zref = np.empty_like(b)
    zref[perm] = np.linalg.solve(Gl, b[perm])
    zo = np.empty_like(b)
    zo[perm] = hchol.solve(hchol.hchol(Gp, root, far, 0.0), b[perm])
    assert np.linalg.norm(z - zref) <= 1e-9 * np.linalg.norm(zref)
    assert np.linalg.norm(z - zo) <= 1e-9 * np.linalg.norm(zo)


@pytest.mark.parametrize("eps", [1e-2, 1e-3, 1e-4, 1e-6])
def test_library_factor_against_oracle(eps):
    """eps > 0: the library and the oracle truncate at different points
    (after every low-rank product against after every block update) but to
    the same blockwise accuracy, so both solves are within a few eps of
    G^{-1} b (relative to the condition of G on this mesh) and of each
    other, and preconditioned CG takes the same number of iterations up to
    one."""
    h = _lib()
    v, t, G, root, perm, far = _setup(8, 16)
    m = h.Mesh(v, t)
    T = h.Tree(m, 0, 16)
    P = h.HChol.from_dense(h.Blocks(T, T, 1.0), G, eps)
    Gp = G[np.ix_(perm, perm)]
    L = hchol.hchol(Gp, root, far, eps)
    b = synth.random_vector(len(t), 13)
    zref = np.linalg.solve(G, b)
    z = P.solve_host(b)
    zo = np.empty_like(b)
    zo[perm] = hchol.solve(L, b[perm])
    e_lib = np.linalg.norm(z - zref) / np.linalg.norm(zref)
    e_orc = np.linalg.norm(zo - zref) / np.linalg.norm(zref)
    print("eps %.0e: library %.2e, oracle %.2e, between %.2e" % (
        eps, e_lib, e_orc, np.linalg.norm(z - zo) / np.linalg.norm(zo)))
    assert e_lib <= 5 * eps and e_orc <= 5 * eps
    assert e_lib <= 4 * e_orc + 1e-12 and e_orc <= 4 * e_lib + 1e-12
    _, it_lib, _ = krylov.pcg(lambda p: G @ p, P.solve_host, b, 1e-10, 500)
    _, it_orc, _ = krylov.pcg(lambda p: Gp @ p, lambda r: hchol.solve(L, r), b[perm], 1e-10, 500)
    assert abs(it_lib - it_orc) <= 1, (it_lib, it_orc)
    info = P.info()
    assert info["n"] == len(t) and info["eps"] == eps
    assert 0 < info["dense_entries"] + info["rk_entries"] < len(t) ** 2


def test_library_iterations_stay_bounded():
    """The point of the preconditioner: with eps fixed, preconditioned CG
    needs a few iterations on meshes of 512 and 2048 triangles while plain CG
    needs more and more (the condition number of G grows like 1/h)."""
    h = _lib()
    its = []
    for s in (8, 16):
        v, t = synth.octa_sphere(s)
        G = oracle.slp_dense(v, t, 4)
        T = h.Tree(h.Mesh(v, t), 0, 16)
        P = h.HChol.from_dense(h.Blocks(T, T, 1.0), G, 1e-2)
        b = synth.random_vector(len(t), 14)
        _, it_pc, _ = krylov.pcg(lambda p: G @ p, P.solve_host, b, 1e-10, 1000)
        _, it_cg, _ = krylov.cg(lambda p: G @ p, b, 1e-10, 1000)
        its.append((it_pc, it_cg))
    print(its)
    assert all(pc <= 10 for pc, _ in its)
    assert its[1][1] > its[0][1] and its[1][1] > 5 * its[1][0]


def test_library_rejects_bad_arguments():
    h = _lib()
    v, t = synth.octa_sphere(4)
    m = h.Mesh(v, t)
    T = h.Tree(m, 0, 8)
    G = oracle.slp_dense(v, t, 4)
    with pytest.raises(h.H2BError):
        h.HChol.from_dense(h.Blocks(T, T, 1.0), G, -1.0)
    with pytest.raises(h.H2BError):
        h.HChol.from_dense(h.Blocks(T, h.Tree(m, 1, 8), 1.0), G, 1e-3)
    # an indefinite matrix has no Cholesky factor
    with pytest.raises(h.H2BError):
        h.HChol.from_dense(h.Blocks(T, T, 1.0), -G, 0.0)
