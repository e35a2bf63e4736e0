// Hierarchical (H-) matrices on one cluster tree for the preconditioner:
// coarsening of a symmetric matrix to a given accuracy and its H-Cholesky
// factorisation, both with truncated low-rank arithmetic (host code).
//
// The paper preconditions its solvers by coarsening the compressed matrix
// and factorising it, G ~ L L^T, with the relative accuracy eps_prc of its
// parameter tables (Section 1; Section 5, Table 1).  Here a block of the
// lower triangle is
//   SUB    subdivided along the cluster tree (a cluster that is not a leaf is
//          split into its two children, a leaf cluster is kept),
//   DENSE  an n_t x n_s array, or
//   RK     a low-rank product U V^T with U (n_t x k) and V (n_s x k).
// Rows and columns are positions in the tree's permutation.  Diagonal blocks
// (t, t) store only their lower children; a dense diagonal block is stored
// in full.  Every truncation keeps the singular values above eps times the
// largest one of that block (blockwise relative accuracy eps).
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "h2b_internal.hpp"

namespace h2b {

struct HNode {
    enum Kind : uint8_t { SUB = 0, DENSE = 1, RK = 2 };
    int t = -1, s = -1;
    Kind kind = SUB;
    int ch[4] = {-1, -1, -1, -1};  // SUB: block (row part i, column part j) at 2 i + j; -1 where absent
    int k = 0;                      // RK: rank
    std::vector<double> a, b;       // DENSE: a (n_t x n_s); RK: a = U, b = V; row-major
};

struct HStats {
    int64_t dense_entries = 0, rk_entries = 0;  // stored doubles
    int64_t dense_blocks = 0, rk_blocks = 0, sub_blocks = 0;
    int max_rank = 0;
    int64_t coarsened = 0;  // subdivided blocks replaced by one low-rank block
    int64_t converted = 0;  // dense leaves replaced by low-rank ones
};

struct HMatrix {
    std::shared_ptr<const Tree> tree;
    std::vector<HNode> nodes;
    int root = -1;
    double eps = 0.0;
    bool factored = false;
    HStats stats;
};

// Structure of the lower triangle from a block tree of (tree x tree): SUB
// nodes down to its leaves, which are empty RK (far) or DENSE (near) blocks
// to be filled by the caller.  Returns the node of every leaf of the lower
// triangle by block index: far_node[b] for far block b, near_node[b] for near
// block b (-1 for blocks of the upper triangle).
std::unique_ptr<HMatrix> hmatrix_structure(const Blocks &B, std::vector<int> &far_node, std::vector<int> &near_node);

// From a dense symmetric matrix A (n x n, row-major, positions of the tree):
// near leaves copied, far leaves truncated to eps.
std::unique_ptr<HMatrix> hmatrix_from_dense(const Blocks &B, const double *A, double eps);

// Coarsening to accuracy eps: low-rank leaves truncated, off-diagonal dense
// leaves made low-rank where that stores fewer values, and, from the leaves
// up, subdivided off-diagonal blocks whose parts are all leaves replaced by
// one truncated low-rank block where that stores fewer values.  Diagonal
// blocks keep their structure.
void hmatrix_coarsen(HMatrix &H, double eps);

// H-Cholesky factorisation in place: H holds L with H ~ L L^T afterwards
// (dense diagonal leaves lower triangular).  Fails with H2B_ENOTSUP when a
// pivot is not positive (the truncated matrix is not positive definite).
void hmatrix_cholesky(HMatrix &H);

// x := (L L^T)^{-1} x on the host for a factored H (x in tree positions).
void hmatrix_solve(const HMatrix &H, double *x);

// y += A x for an unfactored H (symmetric: the lower triangle and its
// transpose), x and y in tree positions.
void hmatrix_symv(const HMatrix &H, const double *x, double *y);

HStats hmatrix_stats(const HMatrix &H);

// The substitutions x := L^{-T} L^{-1} x of a factored H as a program of
// steps, each a set of independent tasks (8 int32 each; the items of row
// tasks 8 int32 each) over one value array:
//   diagonal leaf  y[o + i] = sum_j M[j n + i] y[o + j]     [1] o [2] n [3,4] M
//   coefficients   c[q + p] = sum_j M[j k + p] y[yo + j]    [1] yo [2] len [3,4] M [5] k [6] q
//   rows           y[o + e] -= sum over items of sum_j M(e, j) src[x0 + j]
//                                                           [1] o [2] len [3] item begin [4] item end
//   sum            c[d + p] = sum_q c[s + q k + p], q < np     [1] d [2] s [3] np [5] k
//                  (coefficients of a factor longer than COEF_ROWS rows, computed in pieces)
// item: [0] 0: M(e, j) = A[(r0 + e) ld + j], 1: M(e, j) = A[j ld + r0 + e];
//       [1,2] A  [3] ld  [4] r0  [5] src (0: y, 1: c)  [6] x0  [7] number of j.
// The diagonal leaves store the inverse of their factor (its transpose for
// the forward sweep, so that both read M[j n + i]).  Steps [0, fw_steps)
// are the forward substitution, the rest the backward one.
struct HProgram {
    static constexpr int TW = 8, MAXDIAG = 256;
    static constexpr int COEF_ROWS = 1024;  // rows per coefficient task
    enum : int32_t { T_DIAG = 0, T_COEF = 1, T_ROWS = 2, T_SUM = 3 };
    enum : int32_t { I_ROW = 0, I_COL = 1 };
    std::vector<double> vals;
    std::vector<int32_t> step_ptr{0}, tasks, items;
    int64_t ncoef = 0;
    int fw_steps = 0;
    bool built = false;
};

// Builds the program of a factored H (H2B_ENOTSUP for dense diagonal leaves
// above MAXDIAG rows).
void hprogram_build(const HMatrix &H, HProgram &F);
// Runs it on the host on y (n entries, tree positions), checking every
// index against its array (H2B_EDEVICE when one is out of range).
void hprogram_run(const HProgram &F, int64_t n, double *y);

// Truncation of U (m x k) V^T (n x k) to the singular values above eps times
// the largest; returns the new rank.
int truncate_rk(int m, int n, int k, std::vector<double> &U, std::vector<double> &V, double eps);

// One-sided Jacobi SVD of A (m x n, row-major, m >= n): A = W diag(sigma) Z^T,
// W (m x n), Z (n x n), sigma descending.
void svd_jacobi(int m, int n, const double *A, std::vector<double> &W, std::vector<double> &sigma,
                std::vector<double> &Z);

}  // namespace h2b
