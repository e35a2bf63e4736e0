"""Test infrastructure only: the coarsened H-Cholesky factorisation of a
symmetric positive definite matrix, in plain numpy with every block stored
dense (small matrices only).

The paper preconditions its solvers by coarsening the compressed matrix and
factorising it, A ~ L L^T, in H-matrix arithmetic with a relative accuracy
eps_prc (Section 1; the eps_prc column of the parameter table of Section 5).
Written out on the oracle's own cluster and block trees:

* Truncation of a block B to accuracy eps: its singular value decomposition
  with the singular values not above eps times the largest set to zero.
* Low-rank blocks of the lower triangle: the farfield (admissible) blocks,
  truncated once at the start.  Coarsening: an off-diagonal nearfield leaf
  becomes low-rank when its truncated rank k stores fewer values,
  k (n_t + n_s) < n_t n_s; from the leaves up, an off-diagonal block whose
  parts are all leaves becomes one low-rank block when its truncated rank
  stores no more values than its parts.  Diagonal blocks keep their
  structure.
* Factorisation: the recursive block Cholesky over the diagonal blocks,
  L11 = chol(A11), L21 = A21 L11^{-T}, L22 = chol(A22 - L21 L21^T), with the
  dense Cholesky factorisation at the leaves; after each of the last two
  steps every low-rank block inside the updated block is truncated again.

With eps = 0 nothing is truncated and L is the Cholesky factor of A.  The
matrix is in the cluster order (positions of the tree's permutation)."""
import numpy as np


def truncate(B, eps):
    """B with its singular values <= eps * largest dropped."""
    if B.size == 0:
        return B
    U, s, Vt = np.linalg.svd(B, full_matrices=False)
    if s[0] == 0.0:
        return np.zeros_like(B)
    k = int(np.sum(s > eps * s[0]))
    return (U[:, :k] * s[:k]) @ Vt[:k]


def _rank(B, eps):
    if B.size == 0:
        return 0
    s = np.linalg.svd(B, compute_uv=False)
    return int(np.sum(s > eps * s[0])) if s[0] > 0 else 0


def _children(c):
    return c.children if c.children else [c]


def lowrank_blocks(A, root, far, eps):
    """The low-rank blocks (t, s) of the lower triangle after coarsening A to
    accuracy eps: the admissible leaves, the nearfield leaves that store fewer
    values low-rank, and the merged blocks."""
    near_leaves = set()
    far_set = {(t.id, s.id) for t, s in far}
    low = set()

    def sub(t, s):
        return A[t.begin:t.end, s.begin:s.end]

    def rec(t, s):
        # returns True if (t, s) ends as a leaf (dense or low-rank), with its
        # stored size in `store`
        if (t.id, s.id) in far_set:
            low.add((t, s))
            k = _rank(sub(t, s), eps)
            return True, k * ((t.end - t.begin) + (s.end - s.begin))
        if not t.children and not s.children:
            nt, ns = t.end - t.begin, s.end - s.begin
            if t is not s:
                k = _rank(sub(t, s), eps)
                if k * (nt + ns) < nt * ns:
                    low.add((t, s))
                    return True, k * (nt + ns)
            near_leaves.add((t, s))
            return True, nt * ns
        parts = []
        for i, t2 in enumerate(_children(t)):
            for j, s2 in enumerate(_children(s)):
                if t is s and i < j:
                    continue
                parts.append((t2, s2, rec(t2, s2)))
        if t is s or not all(p[2][0] for p in parts):
            return False, 0
        old = sum(p[2][1] for p in parts)
        k = _rank(sub(t, s), eps)
        new = k * ((t.end - t.begin) + (s.end - s.begin))
        if new <= old:
            for t2, s2, _ in parts:
                low.discard((t2, s2))
            _drop_inside(low, t, s)
            low.add((t, s))
            return True, new
        return False, 0

    rec(root, root)
    return low


def _drop_inside(low, t, s):
    for b in list(low):
        if b[0].begin >= t.begin and b[0].end <= t.end and b[1].begin >= s.begin and b[1].end <= s.end:
            low.discard(b)


def hchol(A, root, far, eps):
    """Lower-triangular L (n x n, dense storage) with A ~ L L^T to the
    blockwise accuracy eps; A in cluster order, root the root cluster, far
    the farfield leaves of the block tree."""
    A = np.array(A, dtype=np.float64)
    low = lowrank_blocks(A, root, far, eps) if eps > 0 else set()
    M = A.copy()

    def retruncate(r0, r1, c0, c1):
        for t, s in low:
            if t.begin >= r0 and t.end <= r1 and s.begin >= c0 and s.end <= c1:
                M[t.begin:t.end, s.begin:s.end] = truncate(M[t.begin:t.end, s.begin:s.end], eps)

    retruncate(0, len(A), 0, len(A))

    def chol(c):
        b, e = c.begin, c.end
        if not c.children:
            M[b:e, b:e] = np.linalg.cholesky(M[b:e, b:e])
            return
        c1, c2 = c.children
        chol(c1)
        L11 = np.tril(M[c1.begin:c1.end, c1.begin:c1.end])
        A21 = M[c2.begin:c2.end, c1.begin:c1.end]
        M[c2.begin:c2.end, c1.begin:c1.end] = np.linalg.solve(L11, A21.T).T
        retruncate(c2.begin, c2.end, c1.begin, c1.end)
        L21 = M[c2.begin:c2.end, c1.begin:c1.end]
        M[c2.begin:c2.end, c2.begin:c2.end] -= L21 @ L21.T
        retruncate(c2.begin, c2.end, c2.begin, c2.end)
        chol(c2)

    chol(root)
    return np.tril(M)


def solve(L, b):
    """(L L^T)^{-1} b."""
    y = np.linalg.solve(L, b)
    return np.linalg.solve(L.T, y)
