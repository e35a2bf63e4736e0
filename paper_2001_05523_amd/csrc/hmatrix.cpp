// H-matrix coarsening and H-Cholesky factorisation (host).  The recursions
// follow the block structure of the cluster tree: a symmetric matrix with
// diagonal block (t, t) split into t1, t2 is factorised as
//   L11 L11^T = A11,   L21 = A21 L11^{-T},   L22 L22^T = A22 - L21 L21^T,
// with every product of blocks formed in low-rank or dense arithmetic and
// every low-rank result truncated to the blockwise accuracy eps.
#include "hmatrix.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <numeric>
#include <unordered_map>

#include "linalg.hpp"

namespace h2b {

namespace {

inline int nparts(const Tree &T, int c) { return T.nchild[c] == 0 ? 1 : 2; }
inline int part(const Tree &T, int c, int i) { return T.nchild[c] == 0 ? c : (i == 0 ? T.child0[c] : T.child1[c]); }

// Y (rows of t) += alpha M X (rows of s), or with trans Y (rows of s) +=
// alpha M^T X (rows of t); X and Y have m columns (leading dimensions ldx,
// ldy).  M is an off-diagonal block.
void hmv(const HMatrix &H, const HNode &M, double alpha, const double *X, int ldx, double *Y, int ldy, int m,
         bool trans)
{
    const Tree &T = *H.tree;
    const int nt = T.size(M.t), ns = T.size(M.s);
    if (M.kind == HNode::DENSE) {
        const double *a = M.a.data();
        if (!trans) {
            for (int i = 0; i < nt; ++i) {
                double *y = Y + (size_t)i * ldy;
                for (int j = 0; j < ns; ++j) {
                    const double v = alpha * a[(size_t)i * ns + j];
                    if (v == 0.0) continue;
                    const double *x = X + (size_t)j * ldx;
                    for (int c = 0; c < m; ++c) y[c] += v * x[c];
                }
            }
        } else {
            for (int i = 0; i < nt; ++i) {
                const double *x = X + (size_t)i * ldx;
                for (int j = 0; j < ns; ++j) {
                    const double v = alpha * a[(size_t)i * ns + j];
                    if (v == 0.0) continue;
                    double *y = Y + (size_t)j * ldy;
                    for (int c = 0; c < m; ++c) y[c] += v * x[c];
                }
            }
        }
        return;
    }
    if (M.kind == HNode::RK) {
        const int k = M.k;
        if (k == 0) return;
        // trans: Y += alpha V (U^T X); else Y += alpha U (V^T X)
        const double *in = trans ? M.a.data() : M.b.data();
        const double *out = trans ? M.b.data() : M.a.data();
        const int nin = trans ? nt : ns, nout = trans ? ns : nt;
        std::vector<double> tmp((size_t)k * m, 0.0);
        for (int j = 0; j < nin; ++j) {
            const double *x = X + (size_t)j * ldx;
            for (int p = 0; p < k; ++p) {
                const double v = in[(size_t)j * k + p];
                double *tp = &tmp[(size_t)p * m];
                for (int c = 0; c < m; ++c) tp[c] += v * x[c];
            }
        }
        for (int i = 0; i < nout; ++i) {
            double *y = Y + (size_t)i * ldy;
            for (int p = 0; p < k; ++p) {
                const double v = alpha * out[(size_t)i * k + p];
                const double *tp = &tmp[(size_t)p * m];
                for (int c = 0; c < m; ++c) y[c] += v * tp[c];
            }
        }
        return;
    }
    const int pt = nparts(T, M.t), ps = nparts(T, M.s);
    for (int i = 0; i < pt; ++i)
        for (int j = 0; j < ps; ++j) {
            const int c = M.ch[2 * i + j];
            if (c < 0) continue;
            const HNode &C = H.nodes[c];
            const int ro = T.begin[C.t] - T.begin[M.t], co = T.begin[C.s] - T.begin[M.s];
            if (!trans)
                hmv(H, C, alpha, X + (size_t)co * ldx, ldx, Y + (size_t)ro * ldy, ldy, m, false);
            else
                hmv(H, C, alpha, X + (size_t)ro * ldx, ldx, Y + (size_t)co * ldy, ldy, m, true);
        }
}

void add_rk(HMatrix &H, HNode &C, double alpha, const double *U, int ldu, const double *W, int ldw, int k);

// C += alpha D, D (n_t x n_s, leading dimension ldd)
void add_dense(HMatrix &H, HNode &C, double alpha, const double *D, int ldd)
{
    const Tree &T = *H.tree;
    const int nt = T.size(C.t), ns = T.size(C.s);
    if (C.kind == HNode::DENSE) {
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) C.a[(size_t)i * ns + j] += alpha * D[(size_t)i * ldd + j];
        return;
    }
    if (C.kind == HNode::RK) {
        // D = I D (rank n_t) or D I (rank n_s), whichever is smaller
        if (nt <= ns) {
            std::vector<double> I((size_t)nt * nt, 0.0), Dt((size_t)ns * nt);
            for (int i = 0; i < nt; ++i) I[(size_t)i * nt + i] = 1.0;
            for (int i = 0; i < nt; ++i)
                for (int j = 0; j < ns; ++j) Dt[(size_t)j * nt + i] = alpha * D[(size_t)i * ldd + j];
            add_rk(H, C, 1.0, I.data(), nt, Dt.data(), nt, nt);
        } else {
            std::vector<double> I((size_t)ns * ns, 0.0), Da((size_t)nt * ns);
            for (int j = 0; j < ns; ++j) I[(size_t)j * ns + j] = 1.0;
            for (int i = 0; i < nt; ++i)
                for (int j = 0; j < ns; ++j) Da[(size_t)i * ns + j] = alpha * D[(size_t)i * ldd + j];
            add_rk(H, C, 1.0, Da.data(), ns, I.data(), ns, ns);
        }
        return;
    }
    const int pt = nparts(T, C.t), ps = nparts(T, C.s);
    for (int i = 0; i < pt; ++i)
        for (int j = 0; j < ps; ++j) {
            const int c = C.ch[2 * i + j];
            if (c < 0) continue;
            HNode &S = H.nodes[c];
            const int ro = T.begin[S.t] - T.begin[C.t], co = T.begin[S.s] - T.begin[C.s];
            add_dense(H, S, alpha, D + (size_t)ro * ldd + co, ldd);
        }
}

// C += alpha U W^T with U (n_t x k) and W (n_s x k)
void add_rk(HMatrix &H, HNode &C, double alpha, const double *U, int ldu, const double *W, int ldw, int k)
{
    if (k == 0 || alpha == 0.0) return;
    const Tree &T = *H.tree;
    const int nt = T.size(C.t), ns = T.size(C.s);
    if (C.kind == HNode::RK) {
        const int K = C.k + k;
        std::vector<double> Un((size_t)nt * K), Vn((size_t)ns * K);
        for (int i = 0; i < nt; ++i) {
            for (int p = 0; p < C.k; ++p) Un[(size_t)i * K + p] = C.a[(size_t)i * C.k + p];
            for (int p = 0; p < k; ++p) Un[(size_t)i * K + C.k + p] = alpha * U[(size_t)i * ldu + p];
        }
        for (int j = 0; j < ns; ++j) {
            for (int p = 0; p < C.k; ++p) Vn[(size_t)j * K + p] = C.b[(size_t)j * C.k + p];
            for (int p = 0; p < k; ++p) Vn[(size_t)j * K + C.k + p] = W[(size_t)j * ldw + p];
        }
        C.k = truncate_rk(nt, ns, K, Un, Vn, H.eps);
        C.a.swap(Un);
        C.b.swap(Vn);
        return;
    }
    if (C.kind == HNode::DENSE) {
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) {
                double s = 0.0;
                for (int p = 0; p < k; ++p) s += U[(size_t)i * ldu + p] * W[(size_t)j * ldw + p];
                C.a[(size_t)i * ns + j] += alpha * s;
            }
        return;
    }
    const int pt = nparts(T, C.t), ps = nparts(T, C.s);
    for (int i = 0; i < pt; ++i)
        for (int j = 0; j < ps; ++j) {
            const int c = C.ch[2 * i + j];
            if (c < 0) continue;
            HNode &S = H.nodes[c];
            const int ro = T.begin[S.t] - T.begin[C.t], co = T.begin[S.s] - T.begin[C.s];
            add_rk(H, S, alpha, U + (size_t)ro * ldu, ldu, W + (size_t)co * ldw, ldw, k);
        }
}

// C += alpha A B^T with C = (t, s), A = (t, r), B = (s, r); A and B are
// off-diagonal blocks of H, C a block of H or a temporary low-rank block.
void gemm(HMatrix &H, HNode &C, double alpha, const HNode &A, const HNode &B)
{
    const Tree &T = *H.tree;
    const int nt = T.size(C.t), ns = T.size(C.s), nr = T.size(A.s);
    if (A.kind == HNode::RK) {
        const int k = A.k;
        if (k == 0) return;
        std::vector<double> W((size_t)ns * k, 0.0);  // B V_a
        hmv(H, B, 1.0, A.b.data(), k, W.data(), k, k, false);
        add_rk(H, C, alpha, A.a.data(), k, W.data(), k, k);
        return;
    }
    if (B.kind == HNode::RK) {
        const int k = B.k;
        if (k == 0) return;
        std::vector<double> W((size_t)nt * k, 0.0);  // A V_b
        hmv(H, A, 1.0, B.b.data(), k, W.data(), k, k, false);
        add_rk(H, C, alpha, W.data(), k, B.a.data(), k, k);
        return;
    }
    if (A.kind == HNode::DENSE && B.kind == HNode::DENSE) {
        std::vector<double> D((size_t)nt * ns);
        gemm_nt(nt, ns, nr, A.a.data(), B.a.data(), D.data());
        add_dense(H, C, alpha, D.data(), ns);
        return;
    }
    if (A.kind == HNode::DENSE || B.kind == HNode::DENSE) {
        // D = A B^T through the subdivided factor times the dense one
        std::vector<double> D((size_t)nt * ns, 0.0);
        if (B.kind == HNode::DENSE) {
            std::vector<double> Bt((size_t)nr * ns);
            for (int j = 0; j < ns; ++j)
                for (int q = 0; q < nr; ++q) Bt[(size_t)q * ns + j] = B.a[(size_t)j * nr + q];
            hmv(H, A, 1.0, Bt.data(), ns, D.data(), ns, ns, false);
        } else {
            std::vector<double> At((size_t)nr * nt), Dt((size_t)ns * nt, 0.0);
            for (int i = 0; i < nt; ++i)
                for (int q = 0; q < nr; ++q) At[(size_t)q * nt + i] = A.a[(size_t)i * nr + q];
            hmv(H, B, 1.0, At.data(), nt, Dt.data(), nt, nt, false);
            for (int i = 0; i < nt; ++i)
                for (int j = 0; j < ns; ++j) D[(size_t)i * ns + j] = Dt[(size_t)j * nt + i];
        }
        add_dense(H, C, alpha, D.data(), ns);
        return;
    }
    // A and B subdivided: over the parts of t, s and r
    const int pt = nparts(T, C.t), ps = nparts(T, C.s), pr = nparts(T, A.s);
    auto a_ch = [&](int i, int q) -> const HNode & { return H.nodes[A.ch[2 * i + q]]; };
    auto b_ch = [&](int j, int q) -> const HNode & { return H.nodes[B.ch[2 * j + q]]; };
    if (C.kind == HNode::SUB) {
        for (int i = 0; i < pt; ++i)
            for (int j = 0; j < ps; ++j) {
                const int c = C.ch[2 * i + j];
                if (c < 0) continue;
                for (int q = 0; q < pr; ++q) gemm(H, H.nodes[c], alpha, a_ch(i, q), b_ch(j, q));
            }
        return;
    }
    if (C.kind == HNode::DENSE || (pt == 1 && ps == 1)) {
        for (int i = 0; i < pt; ++i)
            for (int j = 0; j < ps; ++j)
                for (int q = 0; q < pr; ++q) gemm(H, C, alpha, a_ch(i, q), b_ch(j, q));
        return;
    }
    // low-rank C over split clusters: the products of the parts go into
    // temporary low-rank parts, which are then merged into C and truncated
    HNode tmp[4];
    int K = C.k;
    for (int i = 0; i < pt; ++i)
        for (int j = 0; j < ps; ++j) {
            HNode &P = tmp[2 * i + j];
            P.t = part(T, C.t, i);
            P.s = part(T, C.s, j);
            P.kind = HNode::RK;
            for (int q = 0; q < pr; ++q) gemm(H, P, alpha, a_ch(i, q), b_ch(j, q));
            K += P.k;
        }
    std::vector<double> Un((size_t)nt * K, 0.0), Vn((size_t)ns * K, 0.0);
    for (int i = 0; i < nt; ++i)
        for (int p = 0; p < C.k; ++p) Un[(size_t)i * K + p] = C.a[(size_t)i * C.k + p];
    for (int j = 0; j < ns; ++j)
        for (int p = 0; p < C.k; ++p) Vn[(size_t)j * K + p] = C.b[(size_t)j * C.k + p];
    int col = C.k;
    for (int i = 0; i < pt; ++i)
        for (int j = 0; j < ps; ++j) {
            const HNode &P = tmp[2 * i + j];
            const int ro = T.begin[P.t] - T.begin[C.t], co = T.begin[P.s] - T.begin[C.s];
            const int pn = T.size(P.t), pm = T.size(P.s);
            for (int r = 0; r < pn; ++r)
                for (int p = 0; p < P.k; ++p) Un[(size_t)(ro + r) * K + col + p] = P.a[(size_t)r * P.k + p];
            for (int r = 0; r < pm; ++r)
                for (int p = 0; p < P.k; ++p) Vn[(size_t)(co + r) * K + col + p] = P.b[(size_t)r * P.k + p];
            col += P.k;
        }
    C.k = truncate_rk(nt, ns, K, Un, Vn, H.eps);
    C.a.swap(Un);
    C.b.swap(Vn);
}

// L Y = X in place for the diagonal block L = (s, s); X (n_s x m)
void solve_lower(const HMatrix &H, const HNode &L, double *X, int ldx, int m)
{
    const Tree &T = *H.tree;
    const int n = T.size(L.s);
    if (L.kind == HNode::DENSE) {
        const double *a = L.a.data();
        for (int i = 0; i < n; ++i) {
            double *xi = X + (size_t)i * ldx;
            for (int j = 0; j < i; ++j) {
                const double v = a[(size_t)i * n + j];
                if (v == 0.0) continue;
                const double *xj = X + (size_t)j * ldx;
                for (int c = 0; c < m; ++c) xi[c] -= v * xj[c];
            }
            const double d = 1.0 / a[(size_t)i * n + i];
            for (int c = 0; c < m; ++c) xi[c] *= d;
        }
        return;
    }
    const HNode &L11 = H.nodes[L.ch[0]], &L21 = H.nodes[L.ch[2]], &L22 = H.nodes[L.ch[3]];
    const int n1 = T.size(L11.s);
    solve_lower(H, L11, X, ldx, m);
    hmv(H, L21, -1.0, X, ldx, X + (size_t)n1 * ldx, ldx, m, false);
    solve_lower(H, L22, X + (size_t)n1 * ldx, ldx, m);
}

// L^T Y = X in place
void solve_lower_trans(const HMatrix &H, const HNode &L, double *X, int ldx, int m)
{
    const Tree &T = *H.tree;
    const int n = T.size(L.s);
    if (L.kind == HNode::DENSE) {
        const double *a = L.a.data();
        for (int i = n - 1; i >= 0; --i) {
            double *xi = X + (size_t)i * ldx;
            for (int j = i + 1; j < n; ++j) {
                const double v = a[(size_t)j * n + i];
                if (v == 0.0) continue;
                const double *xj = X + (size_t)j * ldx;
                for (int c = 0; c < m; ++c) xi[c] -= v * xj[c];
            }
            const double d = 1.0 / a[(size_t)i * n + i];
            for (int c = 0; c < m; ++c) xi[c] *= d;
        }
        return;
    }
    const HNode &L11 = H.nodes[L.ch[0]], &L21 = H.nodes[L.ch[2]], &L22 = H.nodes[L.ch[3]];
    const int n1 = T.size(L11.s);
    solve_lower_trans(H, L22, X + (size_t)n1 * ldx, ldx, m);
    hmv(H, L21, -1.0, X + (size_t)n1 * ldx, ldx, X, ldx, m, true);
    solve_lower_trans(H, L11, X, ldx, m);
}

// X := X L^{-T} for the off-diagonal block X = (t, s) and L = (s, s)
void trsm(HMatrix &H, const HNode &L, HNode &X)
{
    const Tree &T = *H.tree;
    const int nt = T.size(X.t), ns = T.size(X.s);
    if (X.kind == HNode::RK) {
        if (X.k > 0) solve_lower(H, L, X.b.data(), X.k, X.k);  // U V^T L^{-T} = U (L^{-1} V)^T
        return;
    }
    if (X.kind == HNode::DENSE) {
        std::vector<double> Xt((size_t)ns * nt);
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) Xt[(size_t)j * nt + i] = X.a[(size_t)i * ns + j];
        solve_lower(H, L, Xt.data(), nt, nt);
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) X.a[(size_t)i * ns + j] = Xt[(size_t)j * nt + i];
        return;
    }
    const int pt = nparts(T, X.t);
    if (T.nchild[X.s] == 0) {
        for (int i = 0; i < pt; ++i) trsm(H, L, H.nodes[X.ch[2 * i]]);
        return;
    }
    const HNode &L11 = H.nodes[L.ch[0]], &L21 = H.nodes[L.ch[2]], &L22 = H.nodes[L.ch[3]];
    for (int i = 0; i < pt; ++i) {
        HNode &X1 = H.nodes[X.ch[2 * i]], &X2 = H.nodes[X.ch[2 * i + 1]];
        trsm(H, L11, X1);
        gemm(H, X2, -1.0, X1, L21);
        trsm(H, L22, X2);
    }
}

void cholesky(HMatrix &H, HNode &L)
{
    const Tree &T = *H.tree;
    if (L.kind == HNode::DENSE) {
        const int n = T.size(L.t);
        double *a = L.a.data();
        for (int j = 0; j < n; ++j) {
            double d = a[(size_t)j * n + j];
            for (int k = 0; k < j; ++k) d -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
            if (!(d > 0.0))
                fail(H2B_ENOTSUP, "H-Cholesky: a pivot is not positive (the matrix truncated to this accuracy is "
                                  "not positive definite; use a smaller eps)");
            const double l = std::sqrt(d);
            a[(size_t)j * n + j] = l;
            for (int i = j + 1; i < n; ++i) {
                double s = a[(size_t)i * n + j];
                for (int k = 0; k < j; ++k) s -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
                a[(size_t)i * n + j] = s / l;
            }
            for (int i = 0; i < j; ++i) a[(size_t)i * n + j] = 0.0;
        }
        return;
    }
    HNode &L11 = H.nodes[L.ch[0]], &L21 = H.nodes[L.ch[2]], &L22 = H.nodes[L.ch[3]];
    cholesky(H, L11);
    trsm(H, L11, L21);
    gemm(H, L22, -1.0, L21, L21);
    cholesky(H, L22);
}

// the matrix D (m x n) as a truncated low-rank product U V^T
int dense_to_rk(int m, int n, const double *D, double eps, std::vector<double> &U, std::vector<double> &V)
{
    std::vector<double> W, sig, Z;
    const bool tr = n > m;
    std::vector<double> A;
    if (tr) {
        A.resize((size_t)n * m);
        for (int i = 0; i < m; ++i)
            for (int j = 0; j < n; ++j) A[(size_t)j * m + i] = D[(size_t)i * n + j];
        svd_jacobi(n, m, A.data(), W, sig, Z);  // D^T = W S Z^T, D = Z S W^T
    } else {
        svd_jacobi(m, n, D, W, sig, Z);  // D = W S Z^T
    }
    const int r = (int)sig.size();
    int k = 0;
    while (k < r && sig[k] > 0.0 && sig[k] > eps * sig[0]) ++k;
    U.assign((size_t)m * k, 0.0);
    V.assign((size_t)n * k, 0.0);
    // left factor (rows m) and right factor (rows n) of D
    const std::vector<double> &Lf = tr ? Z : W, &Rf = tr ? W : Z;
    for (int i = 0; i < m; ++i)
        for (int p = 0; p < k; ++p) U[(size_t)i * k + p] = Lf[(size_t)i * r + p] * sig[p];
    for (int j = 0; j < n; ++j)
        for (int p = 0; p < k; ++p) V[(size_t)j * k + p] = Rf[(size_t)j * r + p];
    return k;
}

void stats_rec(const HMatrix &H, int idx, HStats &S)
{
    const HNode &N = H.nodes[idx];
    const Tree &T = *H.tree;
    if (N.kind == HNode::DENSE) {
        ++S.dense_blocks;
        S.dense_entries += (int64_t)T.size(N.t) * T.size(N.s);
    } else if (N.kind == HNode::RK) {
        ++S.rk_blocks;
        S.rk_entries += (int64_t)N.k * (T.size(N.t) + T.size(N.s));
        S.max_rank = std::max(S.max_rank, N.k);
    } else {
        ++S.sub_blocks;
        for (int c : N.ch)
            if (c >= 0) stats_rec(H, c, S);
    }
}

void symv_rec(const HMatrix &H, const HNode &N, const double *x, double *y)
{
    const Tree &T = *H.tree;
    if (N.t != N.s) {
        const int ro = T.begin[N.t], co = T.begin[N.s];
        hmv(H, N, 1.0, x + co, 1, y + ro, 1, 1, false);
        hmv(H, N, 1.0, x + ro, 1, y + co, 1, 1, true);
        return;
    }
    if (N.kind == HNode::DENSE) {
        const int n = T.size(N.t), o = T.begin[N.t];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) y[o + i] += N.a[(size_t)i * n + j] * x[o + j];
        return;
    }
    for (int c : N.ch)
        if (c >= 0) symv_rec(H, H.nodes[c], x, y);
}

}  // namespace

void svd_jacobi(int m, int n, const double *A, std::vector<double> &W, std::vector<double> &sigma,
                std::vector<double> &Z)
{
    // column-major working copies: the rotations act on columns
    std::vector<double> a((size_t)n * m), z((size_t)n * n, 0.0);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < n; ++j) a[(size_t)j * m + i] = A[(size_t)i * n + j];
    for (int j = 0; j < n; ++j) z[(size_t)j * n + j] = 1.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        bool rotated = false;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double *ap = &a[(size_t)p * m], *aq = &a[(size_t)q * m];
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int i = 0; i < m; ++i) {
                    al += ap[i] * ap[i];
                    be += aq[i] * aq[i];
                    ga += ap[i] * aq[i];
                }
                if (ga == 0.0 || std::fabs(ga) <= 1e-15 * std::sqrt(al * be)) continue;
                rotated = true;
                const double zeta = (be - al) / (2.0 * ga);
                const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
                const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
                for (int i = 0; i < m; ++i) {
                    const double u = ap[i], v = aq[i];
                    ap[i] = c * u - s * v;
                    aq[i] = s * u + c * v;
                }
                double *zp = &z[(size_t)p * n], *zq = &z[(size_t)q * n];
                for (int i = 0; i < n; ++i) {
                    const double u = zp[i], v = zq[i];
                    zp[i] = c * u - s * v;
                    zq[i] = s * u + c * v;
                }
            }
        if (!rotated) break;
    }
    std::vector<double> nrm(n);
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < m; ++i) s += a[(size_t)j * m + i] * a[(size_t)j * m + i];
        nrm[j] = std::sqrt(s);
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return nrm[x] > nrm[y]; });
    W.assign((size_t)m * n, 0.0);
    Z.assign((size_t)n * n, 0.0);
    sigma.assign(n, 0.0);
    for (int jj = 0; jj < n; ++jj) {
        const int j = idx[jj];
        sigma[jj] = nrm[j];
        const double inv = nrm[j] > 0.0 ? 1.0 / nrm[j] : 0.0;
        for (int i = 0; i < m; ++i) W[(size_t)i * n + jj] = a[(size_t)j * m + i] * inv;
        for (int i = 0; i < n; ++i) Z[(size_t)i * n + jj] = z[(size_t)j * n + i];
    }
}

int truncate_rk(int m, int n, int k, std::vector<double> &U, std::vector<double> &V, double eps)
{
    if (k == 0) {
        U.clear();
        V.clear();
        return 0;
    }
    std::vector<double> Q1, R1, Q2, R2;
    householder_qr(m, k, U.data(), Q1, R1);
    householder_qr(n, k, V.data(), Q2, R2);
    const int r1 = std::min(m, k), r2 = std::min(n, k);
    std::vector<double> C((size_t)r1 * r2);
    gemm_nt(r1, r2, k, R1.data(), R2.data(), C.data());  // R1 R2^T
    // C = Wl S Wr^T
    std::vector<double> W, sig, Z, Wl, Wr;
    int r;
    if (r1 >= r2) {
        svd_jacobi(r1, r2, C.data(), W, sig, Z);
        r = r2;
        Wl.swap(W);  // r1 x r2
        Wr.swap(Z);  // r2 x r2
    } else {
        std::vector<double> Ct((size_t)r2 * r1);
        for (int i = 0; i < r1; ++i)
            for (int j = 0; j < r2; ++j) Ct[(size_t)j * r1 + i] = C[(size_t)i * r2 + j];
        svd_jacobi(r2, r1, Ct.data(), W, sig, Z);  // C^T = W S Z^T
        r = r1;
        Wl.swap(Z);  // r1 x r1
        Wr.swap(W);  // r2 x r1
    }
    int l = 0;
    while (l < r && sig[l] > 0.0 && sig[l] > eps * sig[0]) ++l;
    std::vector<double> Un((size_t)m * l, 0.0), Vn((size_t)n * l, 0.0);
    for (int i = 0; i < m; ++i)
        for (int q = 0; q < r1; ++q) {
            const double v = Q1[(size_t)i * r1 + q];
            if (v == 0.0) continue;
            for (int p = 0; p < l; ++p) Un[(size_t)i * l + p] += v * Wl[(size_t)q * r + p] * sig[p];
        }
    for (int j = 0; j < n; ++j)
        for (int q = 0; q < r2; ++q) {
            const double v = Q2[(size_t)j * r2 + q];
            if (v == 0.0) continue;
            for (int p = 0; p < l; ++p) Vn[(size_t)j * l + p] += v * Wr[(size_t)q * r + p];
        }
    U.swap(Un);
    V.swap(Vn);
    return l;
}

std::unique_ptr<HMatrix> hmatrix_structure(const Blocks &B, std::vector<int> &far_node, std::vector<int> &near_node)
{
    if (B.rows != B.cols) fail(H2B_EINVAL, "the H-matrix preconditioner needs one cluster tree for rows and columns");
    const Tree &T = *B.rows;
    auto H = std::make_unique<HMatrix>();
    H->tree = B.rows;
    const int64_t nc = T.nclusters();
    std::unordered_map<int64_t, int> far, near;
    for (size_t b = 0; b < B.far_t.size(); ++b) far[(int64_t)B.far_t[b] * nc + B.far_s[b]] = (int)b;
    for (size_t b = 0; b < B.near_t.size(); ++b) near[(int64_t)B.near_t[b] * nc + B.near_s[b]] = (int)b;
    far_node.assign(B.far_t.size(), -1);
    near_node.assign(B.near_t.size(), -1);
    std::function<int(int, int)> rec = [&](int t, int s) -> int {
        const int idx = (int)H->nodes.size();
        H->nodes.emplace_back();
        H->nodes[idx].t = t;
        H->nodes[idx].s = s;
        const int64_t key = (int64_t)t * nc + s;
        auto f = far.find(key);
        if (f != far.end()) {
            H->nodes[idx].kind = HNode::RK;
            far_node[f->second] = idx;
            return idx;
        }
        auto q = near.find(key);
        if (q != near.end()) {
            H->nodes[idx].kind = HNode::DENSE;
            H->nodes[idx].a.assign((size_t)T.size(t) * T.size(s), 0.0);
            near_node[q->second] = idx;
            return idx;
        }
        if (T.nchild[t] == 0 && T.nchild[s] == 0) fail(H2B_EINVAL, "block tree does not cover a leaf pair");
        const int pt = nparts(T, t), ps = nparts(T, s);
        for (int i = 0; i < pt; ++i)
            for (int j = 0; j < ps; ++j) {
                if (t == s && i < j) continue;  // upper part of a diagonal block
                const int c = rec(part(T, t, i), part(T, s, j));
                H->nodes[idx].ch[2 * i + j] = c;
            }
        return idx;
    };
    H->root = rec(0, 0);
    return H;
}

std::unique_ptr<HMatrix> hmatrix_from_dense(const Blocks &B, const double *A, double eps)
{
    std::vector<int> fn, nn;
    auto H = hmatrix_structure(B, fn, nn);
    H->eps = eps;
    const Tree &T = *H->tree;
    const int64_t n = T.n;
    for (size_t b = 0; b < fn.size(); ++b) {
        if (fn[b] < 0) continue;
        HNode &N = H->nodes[fn[b]];
        const int nt = T.size(N.t), ns = T.size(N.s), r0 = T.begin[N.t], c0 = T.begin[N.s];
        std::vector<double> D((size_t)nt * ns);
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) D[(size_t)i * ns + j] = A[(size_t)(r0 + i) * n + c0 + j];
        N.k = dense_to_rk(nt, ns, D.data(), eps, N.a, N.b);
    }
    for (size_t b = 0; b < nn.size(); ++b) {
        if (nn[b] < 0) continue;
        HNode &N = H->nodes[nn[b]];
        const int nt = T.size(N.t), ns = T.size(N.s), r0 = T.begin[N.t], c0 = T.begin[N.s];
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < ns; ++j) N.a[(size_t)i * ns + j] = A[(size_t)(r0 + i) * n + c0 + j];
    }
    return H;
}

void hmatrix_coarsen(HMatrix &H, double eps)
{
    H.eps = eps;
    const Tree &T = *H.tree;
    // leaves first (independent), then the bottom-up merge
    std::vector<int> leaves;
    for (size_t i = 0; i < H.nodes.size(); ++i) {
        const HNode &N = H.nodes[i];
        if (N.kind != HNode::SUB && N.t != N.s) leaves.push_back((int)i);
    }
    std::vector<char> conv(leaves.size(), 0);
    parallel_for((int64_t)leaves.size(), [&](int64_t q) {
        HNode &N = H.nodes[leaves[q]];
        const int nt = T.size(N.t), ns = T.size(N.s);
        if (N.kind == HNode::RK) {
            N.k = truncate_rk(nt, ns, N.k, N.a, N.b, eps);
        } else {
            std::vector<double> U, V;
            const int k = dense_to_rk(nt, ns, N.a.data(), eps, U, V);
            if ((int64_t)k * (nt + ns) < (int64_t)nt * ns) {
                N.kind = HNode::RK;
                N.k = k;
                N.a.swap(U);
                N.b.swap(V);
                conv[q] = 1;
            }
        }
    });
    for (char c : conv) H.stats.converted += c;
    std::function<void(int)> rec = [&](int idx) {
        if (H.nodes[idx].kind != HNode::SUB) return;
        for (int c : H.nodes[idx].ch)
            if (c >= 0) rec(c);
        HNode &N = H.nodes[idx];
        if (N.t == N.s) return;
        int64_t old = 0;
        int K = 0;
        for (int c : N.ch) {
            if (c < 0) continue;
            const HNode &C = H.nodes[c];
            if (C.kind == HNode::SUB) return;
            const int cn = T.size(C.t), cm = T.size(C.s);
            if (C.kind == HNode::DENSE) {
                old += (int64_t)cn * cm;
                K += std::min(cn, cm);
            } else {
                old += (int64_t)C.k * (cn + cm);
                K += C.k;
            }
        }
        const int nt = T.size(N.t), ns = T.size(N.s);
        std::vector<double> Un((size_t)nt * K, 0.0), Vn((size_t)ns * K, 0.0);
        int col = 0;
        for (int c : N.ch) {
            if (c < 0) continue;
            const HNode &C = H.nodes[c];
            const int ro = T.begin[C.t] - T.begin[N.t], co = T.begin[C.s] - T.begin[N.s];
            const int cn = T.size(C.t), cm = T.size(C.s);
            if (C.kind == HNode::RK) {
                for (int r = 0; r < cn; ++r)
                    for (int p = 0; p < C.k; ++p) Un[(size_t)(ro + r) * K + col + p] = C.a[(size_t)r * C.k + p];
                for (int r = 0; r < cm; ++r)
                    for (int p = 0; p < C.k; ++p) Vn[(size_t)(co + r) * K + col + p] = C.b[(size_t)r * C.k + p];
                col += C.k;
            } else if (cn <= cm) {  // D = I D
                for (int r = 0; r < cn; ++r) Un[(size_t)(ro + r) * K + col + r] = 1.0;
                for (int r = 0; r < cm; ++r)
                    for (int p = 0; p < cn; ++p) Vn[(size_t)(co + r) * K + col + p] = C.a[(size_t)p * cm + r];
                col += cn;
            } else {  // D = D I
                for (int r = 0; r < cn; ++r)
                    for (int p = 0; p < cm; ++p) Un[(size_t)(ro + r) * K + col + p] = C.a[(size_t)r * cm + p];
                for (int r = 0; r < cm; ++r) Vn[(size_t)(co + r) * K + col + r] = 1.0;
                col += cm;
            }
        }
        const int k = truncate_rk(nt, ns, K, Un, Vn, eps);
        if ((int64_t)k * (nt + ns) <= old) {
            N.kind = HNode::RK;
            N.k = k;
            N.a.swap(Un);
            N.b.swap(Vn);
            for (int &c : N.ch) c = -1;
            ++H.stats.coarsened;
        }
    };
    rec(H.root);
    // drop the storage of blocks no longer reachable
    std::vector<char> live(H.nodes.size(), 0);
    std::function<void(int)> mark = [&](int idx) {
        live[idx] = 1;
        for (int c : H.nodes[idx].ch)
            if (c >= 0) mark(c);
    };
    mark(H.root);
    for (size_t i = 0; i < H.nodes.size(); ++i)
        if (!live[i]) {
            std::vector<double>().swap(H.nodes[i].a);
            std::vector<double>().swap(H.nodes[i].b);
        }
}

void hmatrix_cholesky(HMatrix &H)
{
    if (H.factored) fail(H2B_ESTATE, "the H-matrix is already factorised");
    cholesky(H, H.nodes[H.root]);
    H.factored = true;
}

void hmatrix_solve(const HMatrix &H, double *x)
{
    if (!H.factored) fail(H2B_ESTATE, "the H-matrix is not factorised");
    solve_lower(H, H.nodes[H.root], x, 1, 1);
    solve_lower_trans(H, H.nodes[H.root], x, 1, 1);
}

void hmatrix_symv(const HMatrix &H, const double *x, double *y)
{
    if (H.factored) fail(H2B_ESTATE, "the H-matrix is factorised");
    symv_rec(H, H.nodes[H.root], x, y);
}

HStats hmatrix_stats(const HMatrix &H)
{
    HStats S;
    stats_rec(H, H.root, S);
    S.coarsened = H.stats.coarsened;
    S.converted = H.stats.converted;
    return S;
}

// ------------------------------------------------ substitution program

namespace {
constexpr int TW = HProgram::TW, MAXDIAG = HProgram::MAXDIAG;
constexpr int T_DIAG = HProgram::T_DIAG, T_COEF = HProgram::T_COEF, T_ROWS = HProgram::T_ROWS;
constexpr int T_SUM = HProgram::T_SUM;
constexpr int I_ROW = HProgram::I_ROW, I_COL = HProgram::I_COL;

void put64(std::vector<int32_t> &v, size_t at, int64_t x)
{
    v[at] = (int32_t)(uint32_t)(x & 0xffffffffll);
    v[at + 1] = (int32_t)(x >> 32);
}

}  // namespace

void hprogram_build(const HMatrix &H, HProgram &F)
{
    const Tree &T = *H.tree;
    const size_t nn = H.nodes.size();
    // values: diagonal leaves (inverse factor, row-major, and its transpose),
    // off-diagonal dense blocks, low-rank U and V; coefficient slots
    std::vector<int64_t> off_a(nn, -1), off_b(nn, -1), coff(nn, -1);
    std::function<void(int)> place = [&](int idx) {
        const HNode &N = H.nodes[idx];
        if (N.kind == HNode::SUB) {
            for (int c : N.ch)
                if (c >= 0) place(c);
            return;
        }
        const int nt = T.size(N.t), ns = T.size(N.s);
        if (N.t == N.s) {
            if (nt > MAXDIAG) fail(H2B_ENOTSUP, "H-Cholesky: dense diagonal leaves hold at most 256 rows");
            // Linv = L^{-1} by forward substitution on the identity
            std::vector<double> inv((size_t)nt * nt, 0.0);
            for (int c = 0; c < nt; ++c)
                for (int i = c; i < nt; ++i) {
                    double s = (i == c) ? 1.0 : 0.0;
                    for (int j = c; j < i; ++j) s -= N.a[(size_t)i * nt + j] * inv[(size_t)j * nt + c];
                    inv[(size_t)i * nt + c] = s / N.a[(size_t)i * nt + i];
                }
            off_a[idx] = (int64_t)F.vals.size();  // Linv^T (forward: out_i = sum_j Linv^T[j][i] y_j)
            for (int j = 0; j < nt; ++j)
                for (int i = 0; i < nt; ++i) F.vals.push_back(inv[(size_t)i * nt + j]);
            off_b[idx] = (int64_t)F.vals.size();  // Linv (backward)
            F.vals.insert(F.vals.end(), inv.begin(), inv.end());
            return;
        }
        if (N.kind == HNode::DENSE) {
            off_a[idx] = (int64_t)F.vals.size();
            F.vals.insert(F.vals.end(), N.a.begin(), N.a.end());
            return;
        }
        if (N.k == 0) return;
        off_a[idx] = (int64_t)F.vals.size();
        F.vals.insert(F.vals.end(), N.a.begin(), N.a.end());
        off_b[idx] = (int64_t)F.vals.size();
        F.vals.insert(F.vals.end(), N.b.begin(), N.b.end());
        coff[idx] = F.ncoef;
        F.ncoef += N.k;
        (void)ns;
    };
    place(H.root);
    if (F.ncoef > INT32_MAX || (int64_t)T.n > INT32_MAX) fail(H2B_ENOTSUP, "H-Cholesky: problem too large");

    auto leaves_of = [&](int idx, std::vector<int> &out) {
        std::function<void(int)> rec = [&](int i) {
            const HNode &N = H.nodes[i];
            if (N.kind == HNode::SUB) {
                for (int c : N.ch)
                    if (c >= 0) rec(c);
            } else if (N.kind == HNode::DENSE || N.k > 0) {
                out.push_back(i);
            }
        };
        rec(idx);
    };
    auto tree_leaves = [&](int c, std::vector<int> &out) {
        std::function<void(int)> rec = [&](int x) {
            if (T.nchild[x] == 0)
                out.push_back(x);
            else {
                rec(T.child0[x]);
                rec(T.child1[x]);
            }
        };
        rec(c);
    };
    auto end_step = [&] { F.step_ptr.push_back((int32_t)(F.tasks.size() / TW)); };
    auto task = [&]() -> size_t {
        const size_t at = F.tasks.size();
        F.tasks.resize(at + TW, 0);
        return at;
    };
    auto item = [&](int mode, int64_t voff, int ld, int r0, int src, int x0, int nin) {
        const size_t at = F.items.size();
        F.items.resize(at + TW, 0);
        F.items[at] = mode;
        put64(F.items, at + 1, voff);
        F.items[at + 3] = ld;
        F.items[at + 4] = r0;
        F.items[at + 5] = src;
        F.items[at + 6] = x0;
        F.items[at + 7] = nin;
    };
    // update y_rows(X.t) -= X y_cols(X.s) (forward) or y_cols(X.s) -= X^T y_rows(X.t)
    auto update = [&](int xi, bool fw) {
        std::vector<int> lv;
        leaves_of(xi, lv);
        if (lv.empty()) return;
        // coefficients of the low-rank blocks; a long factor is cut into
        // pieces of COEF_ROWS rows with their own partial coefficients,
        // summed in a step of their own
        bool any_rk = false;
        std::vector<std::array<int64_t, 4>> sums;  // destination, first partial, pieces, rank
        for (int i : lv) {
            const HNode &N = H.nodes[i];
            if (N.kind != HNode::RK) continue;
            any_rk = true;
            const int y0 = fw ? T.begin[N.s] : T.begin[N.t];
            const int len = fw ? T.size(N.s) : T.size(N.t);
            const int64_t M = fw ? off_b[i] : off_a[i];
            const int np = (len + HProgram::COEF_ROWS - 1) / HProgram::COEF_ROWS;
            int64_t dst = coff[i];
            if (np > 1) {
                dst = F.ncoef;
                F.ncoef += (int64_t)np * N.k;
                sums.push_back({coff[i], dst, np, N.k});
            }
            for (int q = 0; q < np; ++q) {
                const int r0 = q * HProgram::COEF_ROWS, rl = std::min(HProgram::COEF_ROWS, len - r0);
                const size_t at = task();
                F.tasks[at] = T_COEF;
                F.tasks[at + 1] = y0 + r0;
                F.tasks[at + 2] = rl;
                put64(F.tasks, at + 3, M + (int64_t)r0 * N.k);
                F.tasks[at + 5] = N.k;
                F.tasks[at + 6] = (int32_t)(dst + (int64_t)q * N.k);
            }
        }
        if (any_rk) end_step();
        if (!sums.empty()) {
            for (const auto &u : sums) {
                const size_t at = task();
                F.tasks[at] = T_SUM;
                F.tasks[at + 1] = (int32_t)u[0];
                F.tasks[at + 2] = (int32_t)u[1];
                F.tasks[at + 3] = (int32_t)u[2];
                F.tasks[at + 5] = (int32_t)u[3];
            }
            end_step();
        }
        const HNode &X = H.nodes[xi];
        std::vector<int> rs;
        tree_leaves(fw ? X.t : X.s, rs);
        for (int r : rs) {
            const int rb = T.begin[r], re = T.end[r];
            const int32_t i0 = (int32_t)(F.items.size() / TW);
            for (int i : lv) {
                const HNode &N = H.nodes[i];
                const int c = fw ? N.t : N.s;
                if (T.begin[c] > rb || T.end[c] < re) continue;
                const int r0 = rb - T.begin[c];
                if (N.kind == HNode::DENSE) {
                    if (fw)
                        item(I_ROW, off_a[i], T.size(N.s), r0, 0, T.begin[N.s], T.size(N.s));
                    else
                        item(I_COL, off_a[i], T.size(N.s), r0, 0, T.begin[N.t], T.size(N.t));
                } else {
                    item(I_ROW, fw ? off_a[i] : off_b[i], N.k, r0, 1, (int)coff[i], N.k);
                }
            }
            const int32_t i1 = (int32_t)(F.items.size() / TW);
            if (i1 == i0) continue;
            const size_t at = task();
            F.tasks[at] = T_ROWS;
            F.tasks[at + 1] = rb;
            F.tasks[at + 2] = re - rb;
            F.tasks[at + 3] = i0;
            F.tasks[at + 4] = i1;
        }
        end_step();
    };
    auto diag = [&](int idx, bool fw) {
        const HNode &N = H.nodes[idx];
        const size_t at = task();
        F.tasks[at] = T_DIAG;
        F.tasks[at + 1] = T.begin[N.t];
        F.tasks[at + 2] = T.size(N.t);
        put64(F.tasks, at + 3, fw ? off_a[idx] : off_b[idx]);
        end_step();
    };
    std::function<void(int)> fwd = [&](int idx) {
        const HNode &N = H.nodes[idx];
        if (N.kind == HNode::DENSE) return diag(idx, true);
        fwd(N.ch[0]);
        update(N.ch[2], true);
        fwd(N.ch[3]);
    };
    std::function<void(int)> bwd = [&](int idx) {
        const HNode &N = H.nodes[idx];
        if (N.kind == HNode::DENSE) return diag(idx, false);
        bwd(N.ch[3]);
        update(N.ch[2], false);
        bwd(N.ch[0]);
    };
    fwd(H.root);
    F.fw_steps = (int)F.step_ptr.size() - 1;
    bwd(H.root);
    if (F.ncoef > INT32_MAX) fail(H2B_ENOTSUP, "H-Cholesky: problem too large");
    F.built = true;
}

void hprogram_run(const HProgram &F, int64_t n, double *y)
{
    if (!F.built) fail(H2B_ESTATE, "the preconditioner has no program");
    const int64_t nv = (int64_t)F.vals.size(), nt = (int64_t)F.tasks.size() / TW;
    const int64_t ni = (int64_t)F.items.size() / TW;
    std::vector<double> c((size_t)std::max<int64_t>(F.ncoef, 1), 0.0), buf;
    auto chk = [](bool ok) {
        if (!ok) fail(H2B_EDEVICE, "H-Cholesky program index out of range");
    };
    auto get64 = [](const int32_t *d) { return (int64_t)(uint32_t)d[0] | ((int64_t)d[1] << 32); };
    for (size_t s = 0; s + 1 < F.step_ptr.size(); ++s) {
        chk(F.step_ptr[s] >= 0 && F.step_ptr[s] <= F.step_ptr[s + 1] && F.step_ptr[s + 1] <= nt);
        for (int ti = F.step_ptr[s]; ti < F.step_ptr[s + 1]; ++ti) {
            const int32_t *d = &F.tasks[(size_t)ti * TW];
            if (d[0] == T_DIAG) {
                const int o = d[1], m = d[2];
                const int64_t M = get64(d + 3);
                chk(o >= 0 && m > 0 && m <= MAXDIAG && o + m <= n && M >= 0 && M + (int64_t)m * m <= nv);
                buf.assign(y + o, y + o + m);
                for (int i = 0; i < m; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < m; ++j) acc += F.vals[M + (int64_t)j * m + i] * buf[j];
                    y[o + i] = acc;
                }
            } else if (d[0] == T_COEF) {
                const int yo = d[1], len = d[2], k = d[5], q = d[6];
                const int64_t M = get64(d + 3);
                chk(yo >= 0 && len >= 0 && yo + len <= n && k > 0 && q >= 0 && q + k <= F.ncoef && M >= 0 &&
                    M + (int64_t)len * k <= nv);
                for (int p = 0; p < k; ++p) {
                    double acc = 0.0;
                    for (int j = 0; j < len; ++j) acc += F.vals[M + (int64_t)j * k + p] * y[yo + j];
                    c[q + p] = acc;
                }
            } else if (d[0] == T_SUM) {
                const int dst = d[1], src = d[2], np = d[3], k = d[5];
                chk(dst >= 0 && dst + k <= F.ncoef && src >= 0 && np > 0 && k > 0 &&
                    src + (int64_t)np * k <= F.ncoef);
                for (int p = 0; p < k; ++p) {
                    double acc = 0.0;
                    for (int q = 0; q < np; ++q) acc += c[src + (int64_t)q * k + p];
                    c[dst + p] = acc;
                }
            } else {
                chk(d[0] == T_ROWS);
                const int o = d[1], len = d[2], i0 = d[3], i1 = d[4];
                chk(o >= 0 && len >= 0 && len <= MAXDIAG && o + len <= n && i0 >= 0 && i0 <= i1 && i1 <= ni);
                for (int e = 0; e < len; ++e) {
                    double acc = 0.0;
                    for (int it = i0; it < i1; ++it) {
                        const int32_t *m = &F.items[(size_t)it * TW];
                        const int64_t A = get64(m + 1);
                        const int ld = m[3], r0 = m[4], x0 = m[6], nin = m[7];
                        const bool from_y = m[5] == 0;
                        chk(x0 >= 0 && nin >= 0 && x0 + nin <= (from_y ? n : F.ncoef) && A >= 0 && ld >= 0 && r0 >= 0);
                        if (m[0] == I_ROW) {
                            chk(A + (int64_t)(r0 + e) * ld + nin <= nv && nin <= ld);
                            for (int j = 0; j < nin; ++j)
                                acc += F.vals[A + (int64_t)(r0 + e) * ld + j] * (from_y ? y[x0 + j] : c[x0 + j]);
                        } else {
                            chk(r0 + e < ld && (nin == 0 || A + (int64_t)(nin - 1) * ld + r0 + e < nv));
                            for (int j = 0; j < nin; ++j)
                                acc += F.vals[A + (int64_t)j * ld + r0 + e] * (from_y ? y[x0 + j] : c[x0 + j]);
                        }
                    }
                    y[o + e] -= acc;
                }
            }
        }
    }
}

}  // namespace h2b
