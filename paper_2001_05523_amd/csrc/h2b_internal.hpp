// Internal data structures of the H^2 boundary element library (host side).
#pragma once

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/h2bem.h"

namespace h2b {

// Error carrying a status code; converted to h2b_status at the C boundary.
struct Error : std::runtime_error {
    h2b_status code;
    Error(h2b_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(h2b_status c, const std::string &m) { throw Error(c, m); }

// ------------------------------------------------------------------- mesh

struct Mesh {
    int64_t nv = 0, nt = 0;
    std::vector<double> vx, vy, vz;     // vertex coordinates (SoA)
    std::vector<int32_t> t0, t1, t2;    // triangle corners, counter-clockwise from outside
    std::vector<double> area;           // |tau|
    std::vector<double> nx, ny, nz;     // outward unit normals
    std::vector<double> cx, cy, cz;     // centroids
    std::vector<int64_t> vt_ptr;        // vertex -> adjacent triangles (CSR)
    std::vector<int32_t> vt_idx;
};

// ------------------------------------------------------------------- tree

struct Tree {
    std::shared_ptr<const Mesh> mesh;
    h2b_space space = H2B_P0;
    int leaf = 0;
    int64_t n = 0;
    std::vector<int32_t> perm;          // position -> original index
    std::vector<int32_t> begin, end;    // cluster index ranges (pre-order ids)
    std::vector<int32_t> parent, child0, child1, nchild, level;
    std::vector<double> box;            // 6 per cluster: lo xyz, hi xyz (support box B_t)
    int nlevels = 0;
    std::vector<int32_t> leaves;        // leaf cluster ids in pre-order
    std::vector<std::vector<int32_t>> by_level;  // cluster ids per level

    int64_t nclusters() const { return (int64_t)begin.size(); }
    bool is_leaf(int c) const { return nchild[c] == 0; }
    int size(int c) const { return end[c] - begin[c]; }
    double diam(int c) const;
};

double box_dist(const Tree &a, int t, const Tree &b, int s);

struct Blocks {
    std::shared_ptr<const Tree> rows, cols;
    double eta = 1.0;
    bool far_disabled = false;
    std::vector<int32_t> far_t, far_s;    // farfield leaves
    std::vector<int32_t> near_t, near_s;  // nearfield leaves
};

std::shared_ptr<Mesh> make_mesh(int64_t nv, const double *vx, const double *vy, const double *vz,
                                int64_t nt, const int32_t *t0, const int32_t *t1,
                                const int32_t *t2);
std::shared_ptr<Tree> build_tree(std::shared_ptr<const Mesh> mesh, h2b_space space, int leaf);
std::shared_ptr<Blocks> build_blocks(std::shared_ptr<const Tree> rows,
                                     std::shared_ptr<const Tree> cols, double eta,
                                     bool far_disabled);

// ------------------------------------------------------ numerical helpers

// q-point Gauss-Legendre rule on [0,1] (Golub-Welsch: eigenvalues of the
// symmetric Jacobi matrix of the Legendre recurrence, weights from the first
// eigenvector components).
void gauss_legendre_unit(int q, std::vector<double> &t, std::vector<double> &w);

// Symmetric eigen-decomposition by cyclic Jacobi rotations: a (n x n,
// row-major, overwritten), eigenvalues in ev (descending), eigenvectors as
// columns of z (row-major n x n).
void sym_eig(int n, std::vector<double> &a, std::vector<double> &ev, std::vector<double> &z);

// Chebyshev points (first kind) per axis of the box of cluster c, m per axis.
void cheb_axes(const Tree &tr, int c, int m, double *pts /* 3*m */);

// Green cross approximation on one tree (triangles, or the vertices of K's
// columns): per cluster the rank k_t, the pivots t_hat (original indices,
// pivot order) and V, the leaf basis
// (|t| x k_t, position order) or the stacked transfers [E_1; E_2]
// ((k_1 + k_2) x k_t), both row-major.
struct GcaBases {
    std::vector<int> rank;
    std::vector<std::vector<int32_t>> hat;
    std::vector<std::vector<double>> V;
};
GcaBases gca_bases(const Tree &T, int m, double eps);

}  // namespace h2b
