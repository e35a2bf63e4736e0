// Green cross approximation (GCA, Section 4) of the single-layer matrix G and
// the double-layer matrix K: nested cluster bases by "algebraic
// interpolation" and couplings made of matrix entries,
// A|_{t x s} ~ V_t A|_{t_hat x s_hat} W_s^T.
//
// For every cluster t, bottom-up:
//   1. omega_t = B_t widened by delta_t (the largest side of B_t) on every
//      side, so that dist(boundary of omega_t, B_t) = delta_t (Section 5);
//   2. Green's representation formula on omega_t discretised by an m x m
//      Gauss rule on each face: L = [A C], a_{i nu} = w^{1/2} int psi_i
//      g(x, z_nu), c_{i nu} = w^{1/2} int psi_i dg/dn_z(x, z_nu), for the
//      rows i of t (leaves) or of t_hat_1 followed by t_hat_2 (parents);
//   3. cross approximation of L with full pivoting, stopped when the largest
//      remaining entry is at most eps times the first pivot: row pivots tau,
//      column pivots sigma;
//   4. V = L|_{rows x sigma} (L|_{tau x sigma})^{-1}: the leaf basis V_t, or
//      for a parent the stacked transfer matrices [E_1; E_2]; t_hat = rows[tau].
// The vertex clusters of K's columns take the normal derivative in y of
// Green's formula on omega_s instead (Section 5: K uses the derivatives of the
// approximated kernel): L = [B D], b_{j nu} = w^{1/2} int phi_j(y)
// dg/dn_y(y, z_nu) dy, d_{j nu} = w^{1/2} int phi_j(y) d2g/(dn_y dn_z)(y, z_nu) dy.
// The host builds the bases (clusters of one level in parallel), here; the
// GPU evaluates the coupling entries (gca.hip).
#include <algorithm>
#include <cmath>
#include <vector>

#include "h2b_internal.hpp"
#include "linalg.hpp"

namespace h2b {

namespace {

constexpr double FOUR_PI = 12.566370614359172953850573533118;

struct FaceRule {
    int k = 0;
    std::vector<double> z, n, sw;  // points (3k), outward normals (3k), square roots of the weights
};

// m x m Gauss points on each face of [lo, hi]: axis, then the low side
// before the high side, then the two other axes in increasing order.
FaceRule face_rule(const double *lo, const double *hi, int m, const std::vector<double> &t,
                   const std::vector<double> &w)
{
    FaceRule F;
    F.k = 6 * m * m;
    for (int ax = 0; ax < 3; ++ax) {
        const int o1 = ax == 0 ? 1 : 0, o2 = ax == 2 ? 1 : 2;
        for (int side = 0; side < 2; ++side)
            for (int i = 0; i < m; ++i)
                for (int j = 0; j < m; ++j) {
                    double z[3], n[3] = {0.0, 0.0, 0.0};
                    z[ax] = side ? hi[ax] : lo[ax];
                    z[o1] = lo[o1] + t[i] * (hi[o1] - lo[o1]);
                    z[o2] = lo[o2] + t[j] * (hi[o2] - lo[o2]);
                    n[ax] = side ? 1.0 : -1.0;
                    for (int d = 0; d < 3; ++d) {
                        F.z.push_back(z[d]);
                        F.n.push_back(n[d]);
                    }
                    F.sw.push_back(std::sqrt(w[i] * w[j] * (hi[o1] - lo[o1]) * (hi[o2] - lo[o2])));
                }
    }
    return F;
}

// L = [A C] (rows x 2k, row-major) with the collapsed q x q rule on each triangle.
void green_matrix(const Mesh &M, const std::vector<int32_t> &rows, const FaceRule &F, const std::vector<double> &tq,
                  const std::vector<double> &wq, std::vector<double> &L)
{
    const int k = F.k, q = (int)tq.size();
    L.assign(rows.size() * 2 * (size_t)k, 0.0);
    for (size_t r = 0; r < rows.size(); ++r) {
        const int i = rows[r];
        const int a = M.t0[i], b = M.t1[i], c = M.t2[i];
        const double P0[3] = {M.vx[a], M.vy[a], M.vz[a]}, P1[3] = {M.vx[b], M.vy[b], M.vz[b]},
                     P2[3] = {M.vx[c], M.vy[c], M.vz[c]};
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) e1[d] = P1[d] - P0[d], e2[d] = P2[d] - P1[d];
        const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                     cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double jac = std::sqrt(cx * cx + cy * cy + cz * cz);
        double *row = &L[r * 2 * (size_t)k];
        for (int qa = 0; qa < q; ++qa)
            for (int qb = 0; qb < q; ++qb) {
                const double u1 = tq[qa], u2 = tq[qa] * tq[qb], wt = wq[qa] * wq[qb] * tq[qa] * jac;
                double x[3];
                for (int d = 0; d < 3; ++d) x[d] = P0[d] + u1 * e1[d] + u2 * e2[d];
                for (int nu = 0; nu < k; ++nu) {
                    const double dx = x[0] - F.z[3 * nu], dy = x[1] - F.z[3 * nu + 1], dz = x[2] - F.z[3 * nu + 2];
                    const double r2 = dx * dx + dy * dy + dz * dz, rr = std::sqrt(r2);
                    const double g = 1.0 / (FOUR_PI * rr);
                    const double dn = (dx * F.n[3 * nu] + dy * F.n[3 * nu + 1] + dz * F.n[3 * nu + 2]) * g / r2;
                    row[nu] += wt * g;
                    row[k + nu] += wt * dn;
                }
            }
        for (int nu = 0; nu < k; ++nu) {
            row[nu] *= F.sw[nu];
            row[k + nu] *= F.sw[nu];
        }
    }
}

// L = [B D] for the vertices `rows` (hat functions on the triangles around
// each vertex, normal derivatives in y).  Every triangle around the rows is
// integrated once; its kernel values at the quadrature points go to each of
// its corners that is a row, weighted by that corner's barycentric
// coordinate.  Rows accumulate their triangles in increasing index order.
void green_matrix_p1(const Mesh &M, const std::vector<int32_t> &rows, const FaceRule &F,
                     const std::vector<double> &tq, const std::vector<double> &wq, std::vector<double> &L)
{
    const int k = F.k, q = (int)tq.size(), nq = q * q;
    L.assign(rows.size() * 2 * (size_t)k, 0.0);
    std::vector<std::pair<int32_t, int32_t>> vr(rows.size());
    for (size_t r = 0; r < rows.size(); ++r) vr[r] = {rows[r], (int32_t)r};
    std::sort(vr.begin(), vr.end());
    auto row_of = [&](int32_t v) {
        auto it = std::lower_bound(vr.begin(), vr.end(), std::make_pair(v, (int32_t)-1));
        return it != vr.end() && it->first == v ? it->second : -1;
    };
    std::vector<int32_t> tris;
    for (int32_t v : rows)
        for (int64_t e = M.vt_ptr[v]; e < M.vt_ptr[v + 1]; ++e) tris.push_back(M.vt_idx[e]);
    std::sort(tris.begin(), tris.end());
    tris.erase(std::unique(tris.begin(), tris.end()), tris.end());
    std::vector<double> kb((size_t)nq * k), kd((size_t)nq * k), wp(nq), lam(3 * (size_t)nq);
    for (int32_t i : tris) {
        const int a = M.t0[i], b = M.t1[i], c = M.t2[i];
        const double P0[3] = {M.vx[a], M.vy[a], M.vz[a]}, P1[3] = {M.vx[b], M.vy[b], M.vz[b]},
                     P2[3] = {M.vx[c], M.vy[c], M.vz[c]};
        double e1[3], e2[3];
        for (int d = 0; d < 3; ++d) e1[d] = P1[d] - P0[d], e2[d] = P2[d] - P1[d];
        const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                     cz = e1[0] * e2[1] - e1[1] * e2[0];
        const double jac = std::sqrt(cx * cx + cy * cy + cz * cz);
        const double ny[3] = {cx / jac, cy / jac, cz / jac};
        for (int qa = 0; qa < q; ++qa)
            for (int qb = 0; qb < q; ++qb) {
                const int pt = qa * q + qb;
                const double u1 = tq[qa], u2 = tq[qa] * tq[qb];
                wp[pt] = wq[qa] * wq[qb] * tq[qa] * jac;
                lam[3 * pt] = 1.0 - u1;
                lam[3 * pt + 1] = u1 - u2;
                lam[3 * pt + 2] = u2;
                double y[3];
                for (int d = 0; d < 3; ++d) y[d] = P0[d] + u1 * e1[d] + u2 * e2[d];
                for (int nu = 0; nu < k; ++nu) {
                    const double dx = y[0] - F.z[3 * nu], dy = y[1] - F.z[3 * nu + 1], dz = y[2] - F.z[3 * nu + 2];
                    const double r2 = dx * dx + dy * dy + dz * dz, rr = std::sqrt(r2);
                    const double g3 = 1.0 / (FOUR_PI * rr * r2);  // 1 / (4 pi r^3)
                    const double dny = dx * ny[0] + dy * ny[1] + dz * ny[2];
                    const double *n = &F.n[3 * nu];
                    const double dnz = dx * n[0] + dy * n[1] + dz * n[2];
                    const double nn = ny[0] * n[0] + ny[1] * n[1] + ny[2] * n[2];
                    kb[(size_t)pt * k + nu] = -dny * g3;
                    kd[(size_t)pt * k + nu] = nn * g3 - 3.0 * dny * dnz * g3 / r2;
                }
            }
        const int corners[3] = {a, b, c};
        for (int cc = 0; cc < 3; ++cc) {
            const int r = row_of(corners[cc]);
            if (r < 0) continue;
            double *row = &L[(size_t)r * 2 * k];
            for (int pt = 0; pt < nq; ++pt) {
                const double wl = wp[pt] * lam[3 * pt + cc];
                const double *pb = &kb[(size_t)pt * k], *pd = &kd[(size_t)pt * k];
                for (int nu = 0; nu < k; ++nu) {
                    row[nu] += wl * pb[nu];
                    row[k + nu] += wl * pd[nu];
                }
            }
        }
    }
    for (size_t r = 0; r < rows.size(); ++r) {
        double *row = &L[r * 2 * (size_t)k];
        for (int nu = 0; nu < k; ++nu) {
            row[nu] *= F.sw[nu];
            row[k + nu] *= F.sw[nu];
        }
    }
}

// Cross approximation with full pivoting of R (nr x nc, row-major, consumed).
void aca_full(int nr, int nc, std::vector<double> &R, double eps, std::vector<int> &tau, std::vector<int> &sigma)
{
    tau.clear();
    sigma.clear();
    double first = -1.0;
    for (int step = 0; step < std::min(nr, nc); ++step) {
        int bi = 0, bj = 0;
        double best = -1.0;
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j) {
                const double v = std::fabs(R[(size_t)i * nc + j]);
                if (v > best) best = v, bi = i, bj = j;
            }
        if (first < 0.0) {
            first = best;
            if (first == 0.0) break;
        } else if (best <= eps * first) {
            break;
        }
        tau.push_back(bi);
        sigma.push_back(bj);
        const double piv = R[(size_t)bi * nc + bj];
        std::vector<double> col(nr), row(R.begin() + (size_t)bi * nc, R.begin() + (size_t)(bi + 1) * nc);
        for (int i = 0; i < nr; ++i) col[i] = R[(size_t)i * nc + bj] / piv;
        for (int i = 0; i < nr; ++i)
            for (int j = 0; j < nc; ++j) R[(size_t)i * nc + j] -= col[i] * row[j];
    }
}

// X (nr x k) = B (nr x k) A^{-1}: Gaussian elimination with partial pivoting
// on A^T X^T = B^T.
void solve_right(int k, const std::vector<double> &A, int nr, const std::vector<double> &B, std::vector<double> &X)
{
    std::vector<double> T((size_t)k * k), Y((size_t)k * nr);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) T[(size_t)i * k + j] = A[(size_t)j * k + i];
    for (int i = 0; i < k; ++i)
        for (int r = 0; r < nr; ++r) Y[(size_t)i * nr + r] = B[(size_t)r * k + i];
    for (int c = 0; c < k; ++c) {
        int p = c;
        for (int i = c + 1; i < k; ++i)
            if (std::fabs(T[(size_t)i * k + c]) > std::fabs(T[(size_t)p * k + c])) p = i;
        if (T[(size_t)p * k + c] == 0.0) fail(H2B_EDEVICE, "singular pivot block in the cross approximation");
        if (p != c) {
            for (int j = 0; j < k; ++j) std::swap(T[(size_t)c * k + j], T[(size_t)p * k + j]);
            for (int r = 0; r < nr; ++r) std::swap(Y[(size_t)c * nr + r], Y[(size_t)p * nr + r]);
        }
        for (int i = c + 1; i < k; ++i) {
            const double f = T[(size_t)i * k + c] / T[(size_t)c * k + c];
            if (f == 0.0) continue;
            for (int j = c; j < k; ++j) T[(size_t)i * k + j] -= f * T[(size_t)c * k + j];
            for (int r = 0; r < nr; ++r) Y[(size_t)i * nr + r] -= f * Y[(size_t)c * nr + r];
        }
    }
    for (int c = k - 1; c >= 0; --c) {
        for (int j = c + 1; j < k; ++j) {
            const double f = T[(size_t)c * k + j];
            for (int r = 0; r < nr; ++r) Y[(size_t)c * nr + r] -= f * Y[(size_t)j * nr + r];
        }
        for (int r = 0; r < nr; ++r) Y[(size_t)c * nr + r] /= T[(size_t)c * k + c];
    }
    X.assign((size_t)nr * k, 0.0);
    for (int r = 0; r < nr; ++r)
        for (int i = 0; i < k; ++i) X[(size_t)r * k + i] = Y[(size_t)i * nr + r];
}

}  // namespace

GcaBases gca_bases(const Tree &T, int m, double eps)
{
    const Mesh &M = *T.mesh;
    const int64_t nc = T.nclusters();
    GcaBases G;
    G.rank.assign(nc, 0);
    G.hat.assign(nc, {});
    G.V.assign(nc, {});
    std::vector<double> t, w, tq, wq;
    gauss_legendre_unit(m, t, w);
    gauss_legendre_unit(m + 2, tq, wq);
    for (int lev = T.nlevels - 1; lev >= 0; --lev) {
        const std::vector<int32_t> &cl = T.by_level[lev];
        parallel_for((int64_t)cl.size(), [&](int64_t idx) {
            const int c = cl[idx];
            std::vector<int32_t> rows;
            if (T.nchild[c] == 0) {
                for (int p = T.begin[c]; p < T.end[c]; ++p) rows.push_back(T.perm[p]);
            } else {
                for (int ch : {T.child0[c], T.child1[c]}) rows.insert(rows.end(), G.hat[ch].begin(), G.hat[ch].end());
            }
            const double *bx = &T.box[6 * (size_t)c];
            double delta = 0.0;
            for (int d = 0; d < 3; ++d) delta = std::max(delta, bx[3 + d] - bx[d]);
            const double lo[3] = {bx[0] - delta, bx[1] - delta, bx[2] - delta};
            const double hi[3] = {bx[3] + delta, bx[4] + delta, bx[5] + delta};
            const FaceRule F = face_rule(lo, hi, m, t, w);
            std::vector<double> L;
            if (T.space == H2B_P1)
                green_matrix_p1(M, rows, F, tq, wq, L);
            else
                green_matrix(M, rows, F, tq, wq, L);
            const int nr = (int)rows.size(), ncol = 2 * F.k;
            std::vector<double> R = L;
            std::vector<int> tau, sigma;
            aca_full(nr, ncol, R, eps, tau, sigma);
            const int kk = (int)tau.size();
            std::vector<double> Ats((size_t)kk * kk), Ls((size_t)nr * kk);
            for (int i = 0; i < kk; ++i)
                for (int j = 0; j < kk; ++j) Ats[(size_t)i * kk + j] = L[(size_t)tau[i] * ncol + sigma[j]];
            for (int r = 0; r < nr; ++r)
                for (int j = 0; j < kk; ++j) Ls[(size_t)r * kk + j] = L[(size_t)r * ncol + sigma[j]];
            if (kk > 0) solve_right(kk, Ats, nr, Ls, G.V[c]);
            G.rank[c] = kk;
            G.hat[c].resize(kk);
            for (int i = 0; i < kk; ++i) G.hat[c][i] = rows[tau[i]];
        });
    }
    return G;
}

}  // namespace h2b
