// Host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer:
// mesh checks, cluster and block trees, Chebyshev points, Gauss rules, the
// eigen and QR routines of the recompression, and the Green cross
// approximation's host construction, on octahedral spheres and flat plates of
// several sizes and leaf sizes, plus the rejected inputs.  Built and run by
// tests/test_host_sanitizers.py with g++ (no device code); exits non-zero on
// the first failed check, and the sanitizers abort on the first fault.
#include <cmath>
#include <cstdio>
#include <map>
#include <tuple>
#include <vector>

#include "h2b_internal.hpp"
#include "hmatrix.hpp"
#include "linalg.hpp"

using namespace h2b;

namespace {

int failures = 0;

void check(bool ok, const char *what)
{
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

struct HostMesh {
    std::vector<double> vx, vy, vz;
    std::vector<int32_t> t0, t1, t2;
};

// Octahedron faces split s x s, vertices projected onto the unit sphere,
// triangles counter-clockwise seen from outside.
HostMesh octa_sphere(int s)
{
    HostMesh M;
    std::map<std::tuple<int, int, int>, int32_t> id;
    auto vertex = [&](int a, int b, int c) {
        auto key = std::make_tuple(a, b, c);
        auto it = id.find(key);
        if (it != id.end()) return it->second;
        const double n = std::sqrt(double(a) * a + double(b) * b + double(c) * c);
        M.vx.push_back(a / n);
        M.vy.push_back(b / n);
        M.vz.push_back(c / n);
        const int32_t v = (int32_t)M.vx.size() - 1;
        id[key] = v;
        return v;
    };
    for (int sx : {-1, 1})
        for (int sy : {-1, 1})
            for (int sz : {-1, 1})
                for (int i = 0; i < s; ++i)
                    for (int j = 0; i + j < s; ++j) {
                        // lattice points (x, y, z) with |x| + |y| + |z| = s on this face
                        auto P = [&](int a, int b) { return vertex(sx * a, sy * b, sz * (s - a - b)); };
                        int tri[2][3] = {{P(i, j), P(i + 1, j), P(i, j + 1)}, {0, 0, 0}};
                        int ntri = 1;
                        if (i + j + 1 < s) {
                            tri[1][0] = P(i + 1, j);
                            tri[1][1] = P(i + 1, j + 1);
                            tri[1][2] = P(i, j + 1);
                            ntri = 2;
                        }
                        for (int q = 0; q < ntri; ++q) {
                            int a = tri[q][0], b = tri[q][1], c = tri[q][2];
                            const double e1[3] = {M.vx[b] - M.vx[a], M.vy[b] - M.vy[a], M.vz[b] - M.vz[a]};
                            const double e2[3] = {M.vx[c] - M.vx[a], M.vy[c] - M.vy[a], M.vz[c] - M.vz[a]};
                            const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                                                 e1[0] * e2[1] - e1[1] * e2[0]};
                            if (n[0] * M.vx[a] + n[1] * M.vy[a] + n[2] * M.vz[a] < 0) std::swap(b, c);
                            M.t0.push_back(a);
                            M.t1.push_back(b);
                            M.t2.push_back(c);
                        }
                    }
    return M;
}

// n x n squares of a bent plate, two triangles each.
HostMesh plate(int n)
{
    HostMesh M;
    for (int j = 0; j <= n; ++j)
        for (int i = 0; i <= n; ++i) {
            const double x = double(i) / n, y = double(j) / n;
            M.vx.push_back(x);
            M.vy.push_back(y);
            M.vz.push_back(0.2 * x * x);
        }
    auto v = [&](int i, int j) { return (int32_t)(j * (n + 1) + i); };
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            M.t0.push_back(v(i, j));
            M.t1.push_back(v(i + 1, j));
            M.t2.push_back(v(i + 1, j + 1));
            M.t0.push_back(v(i, j));
            M.t1.push_back(v(i + 1, j + 1));
            M.t2.push_back(v(i, j + 1));
        }
    return M;
}

std::shared_ptr<Mesh> to_mesh(const HostMesh &H)
{
    return make_mesh((int64_t)H.vx.size(), H.vx.data(), H.vy.data(), H.vz.data(), (int64_t)H.t0.size(), H.t0.data(),
                     H.t1.data(), H.t2.data());
}

void check_tree(const Tree &T, int64_t n, int leaf)
{
    check(T.n == n, "tree size");
    std::vector<int> seen(n, 0);
    for (int32_t p : T.perm) ++seen.at(p);
    bool perm_ok = true;
    for (int s : seen) perm_ok = perm_ok && s == 1;
    check(perm_ok, "permutation");
    for (int c : T.leaves) check(T.size(c) <= leaf || T.nchild[c] == 0, "leaf size");
    for (int64_t c = 0; c < T.nclusters(); ++c) {
        if (T.nchild[c] == 0) continue;
        check(T.begin[T.child0[c]] == T.begin[c] && T.end[T.child1[c]] == T.end[c], "children cover the parent");
        double pts[18];
        cheb_axes(T, (int)c, 6, pts);
        for (double p : pts) check(std::isfinite(p), "Chebyshev points finite");
    }
}

void check_blocks(const Blocks &B)
{
    const Tree &R = *B.rows, &C = *B.cols;
    // every (row, column) entry is covered exactly once by the leaves
    std::vector<int> cover((size_t)R.n * C.n, 0);
    auto mark = [&](int t, int s) {
        for (int i = R.begin[t]; i < R.end[t]; ++i)
            for (int j = C.begin[s]; j < C.end[s]; ++j) ++cover[(size_t)i * C.n + j];
    };
    for (size_t b = 0; b < B.far_t.size(); ++b) mark(B.far_t[b], B.far_s[b]);
    for (size_t b = 0; b < B.near_t.size(); ++b) mark(B.near_t[b], B.near_s[b]);
    bool ok = true;
    for (int c : cover) ok = ok && c == 1;
    check(ok, "block leaves cover the matrix once");
}

void check_gca(const Tree &T, int m, double eps)
{
    const GcaBases G = gca_bases(T, m, eps);
    check((int64_t)G.rank.size() == T.nclusters(), "GCA ranks");
    for (int64_t c = 0; c < T.nclusters(); ++c) {
        check((int)G.hat[c].size() == G.rank[c], "GCA pivots");
        const int rows = T.nchild[c] == 0 ? T.size((int)c) : G.rank[T.child0[c]] + G.rank[T.child1[c]];
        check(G.V[c].size() == (size_t)rows * G.rank[c] || G.rank[c] == 0, "GCA basis size");
        for (double v : G.V[c]) check(std::isfinite(v), "GCA basis finite");
    }
}

// H-matrix coarsening, H-Cholesky and the substitution program on a
// symmetric positive definite kernel matrix exp(-|c_i - c_j| / 0.3) + shift I
// over the triangle centroids: the program's solve equals the recursive one,
// and eps = 0 solves exactly.
int check_hchol(const Mesh &M, std::shared_ptr<Tree> T, double eps, double shift = 1e-3)
{
    const int n = (int)T->n;
    std::vector<double> A((size_t)n * n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const int a = T->perm[i], b = T->perm[j];
            const double dx = M.cx[a] - M.cx[b], dy = M.cy[a] - M.cy[b], dz = M.cz[a] - M.cz[b];
            A[(size_t)i * n + j] = std::exp(-std::sqrt(dx * dx + dy * dy + dz * dz) / 0.3) + (i == j ? shift : 0.0);
        }
    auto B = build_blocks(T, T, 1.0, false);
    auto H = hmatrix_from_dense(*B, A.data(), eps);
    hmatrix_coarsen(*H, eps);
    hmatrix_cholesky(*H);
    HProgram P;
    hprogram_build(*H, P);
    std::vector<double> x(n), b(n, 0.0);
    for (int i = 0; i < n; ++i) x[i] = std::sin(0.37 * i + 1.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) b[i] += A[(size_t)i * n + j] * x[j];
    std::vector<double> z1 = b, z2 = b;
    hmatrix_solve(*H, z1.data());
    hprogram_run(P, n, z2.data());
    double d = 0, e = 0, nx = 0;
    for (int i = 0; i < n; ++i) {
        d = std::fmax(d, std::fabs(z1[i] - z2[i]));
        e += (z1[i] - x[i]) * (z1[i] - x[i]);
        nx += x[i] * x[i];
    }
    check(d <= 1e-9 * std::sqrt(nx), "program solve equals the recursive solve");
    if (eps == 0.0) check(std::sqrt(e / nx) <= 1e-8, "exact H-Cholesky solves exactly");
    int sums = 0;
    for (size_t t = 0; t < P.tasks.size(); t += HProgram::TW) sums += P.tasks[t] == HProgram::T_SUM;
    return sums;
}

}  // namespace

int main()
{
    // numerical helpers
    for (int q = 1; q <= 16; ++q) {
        std::vector<double> t, w;
        gauss_legendre_unit(q, t, w);
        double s = 0;
        for (double x : w) s += x;
        check(std::fabs(s - 1.0) < 1e-13, "Gauss weights sum to 1");
    }
    for (int n : {1, 2, 7, 64}) {
        std::vector<double> a((size_t)n * n), ev, z;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) a[(size_t)i * n + j] = 1.0 / (1 + i + j);
        sym_eig(n, a, ev, z);
        check((int)ev.size() == n, "eigenvalues");
        std::vector<double> A((size_t)(n + 3) * n), Q, Rm;
        for (size_t e = 0; e < A.size(); ++e) A[e] = std::sin(0.7 * e + 1.0);
        householder_qr(n + 3, n, A.data(), Q, Rm);
        check(Q.size() == (size_t)(n + 3) * n && Rm.size() == (size_t)n * n, "QR shapes");
    }
    // meshes, trees, blocks
    for (int s : {1, 2, 4, 8, 16}) {
        auto M = to_mesh(octa_sphere(s));
        for (int leaf : {1, 5, 16, 64}) {
            auto R = build_tree(M, H2B_P0, leaf);
            auto C = build_tree(M, H2B_P1, leaf);
            check_tree(*R, M->nt, leaf);
            check_tree(*C, M->nv, leaf);
            if (s <= 8) {
                check_blocks(*build_blocks(R, R, 1.0, false));
                check_blocks(*build_blocks(R, C, 1.0, false));
                check_blocks(*build_blocks(R, C, 0.5, true));
            }
            if (s >= 4 && leaf >= 16) {
                check_gca(*R, 2, 1e-2);
                check_gca(*C, 3, 1e-4);
            }
        }
    }
    for (int leaf : {5, 16})
        for (double eps : {0.0, 1e-4, 1e-2}) {
            auto M = to_mesh(octa_sphere(6));
            check_hchol(*M, build_tree(M, H2B_P0, leaf), eps);
        }
    {
        // 4,232 triangles: coarsened low-rank factors longer than one
        // coefficient piece (none below about 4,000 triangles; a larger shift
        // keeps the matrix truncated to 1e-2 definite)
        auto M = to_mesh(octa_sphere(23));
        check(check_hchol(*M, build_tree(M, H2B_P0, 32), 1e-2, 1.0) > 0, "coefficients computed in pieces");
    }
    {
        auto M = to_mesh(plate(12));
        auto R = build_tree(M, H2B_P0, 8);
        auto C = build_tree(M, H2B_P1, 8);
        check_tree(*R, M->nt, 8);
        check_blocks(*build_blocks(R, C, 1.0, false));
        check_gca(*R, 2, 1e-3);
    }
    // rejected inputs: each must throw, none may touch memory out of bounds
    int rejected = 0;
    auto expect_fail = [&](auto &&f) {
        try {
            f();
        } catch (const Error &) {
            ++rejected;
        }
    };
    HostMesh H = octa_sphere(2);
    expect_fail([&] { make_mesh(2, H.vx.data(), H.vy.data(), H.vz.data(), 1, H.t0.data(), H.t1.data(), H.t2.data()); });
    HostMesh bad = H;
    bad.t1[3] = (int32_t)bad.vx.size();
    expect_fail([&] { to_mesh(bad); });
    bad = H;
    bad.t2[0] = bad.t0[0];
    expect_fail([&] { to_mesh(bad); });
    bad = H;
    bad.vx[0] = NAN;
    expect_fail([&] { to_mesh(bad); });
    auto M = to_mesh(H);
    expect_fail([&] { build_tree(M, H2B_P0, 0); });
    auto R = build_tree(M, H2B_P0, 4);
    auto C = build_tree(M, H2B_P1, 4);
    expect_fail([&] { build_blocks(R, C, 0.0, false); });
    expect_fail([&] { build_blocks(C, R, 1.0, false); });
    check(rejected == 7, "every invalid input rejected");
    if (failures) {
        std::printf("%d checks failed\n", failures);
        return 1;
    }
    std::printf("host checks passed\n");
    return 0;
}
