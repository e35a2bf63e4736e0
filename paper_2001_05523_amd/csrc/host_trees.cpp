// Host-side geometry: mesh checks, cluster trees, block trees, Chebyshev
// points, Gauss-Legendre rules and a small symmetric eigensolver.
#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>

#include "h2b_internal.hpp"

namespace h2b {

// ---------------------------------------------------------------- mesh

std::shared_ptr<Mesh> make_mesh(int64_t nv, const double *vx, const double *vy, const double *vz,
                                int64_t nt, const int32_t *t0, const int32_t *t1,
                                const int32_t *t2)
{
    if (nv < 3 || nt < 1) fail(H2B_EINVAL, "mesh needs nv >= 3 and nt >= 1");
    if (!vx || !vy || !vz || !t0 || !t1 || !t2) fail(H2B_EINVAL, "mesh array is NULL");
    if (nv > INT32_MAX || nt > INT32_MAX) fail(H2B_EINVAL, "mesh too large for 32-bit indices");
    auto m = std::make_shared<Mesh>();
    m->nv = nv;
    m->nt = nt;
    m->vx.assign(vx, vx + nv);
    m->vy.assign(vy, vy + nv);
    m->vz.assign(vz, vz + nv);
    for (int64_t i = 0; i < nv; ++i)
        if (!std::isfinite(vx[i]) || !std::isfinite(vy[i]) || !std::isfinite(vz[i]))
            fail(H2B_EINVAL, "vertex " + std::to_string(i) + " has a non-finite coordinate");
    m->t0.assign(t0, t0 + nt);
    m->t1.assign(t1, t1 + nt);
    m->t2.assign(t2, t2 + nt);
    m->area.resize(nt);
    m->nx.resize(nt);
    m->ny.resize(nt);
    m->nz.resize(nt);
    m->cx.resize(nt);
    m->cy.resize(nt);
    m->cz.resize(nt);
    std::vector<int64_t> deg(nv + 1, 0);
    for (int64_t i = 0; i < nt; ++i) {
        int32_t a = t0[i], b = t1[i], c = t2[i];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv)
            fail(H2B_EINVAL, "triangle " + std::to_string(i) + " has a vertex index out of range");
        if (a == b || b == c || a == c)
            fail(H2B_EINVAL, "triangle " + std::to_string(i) + " repeats a vertex");
        double e1[3] = {vx[b] - vx[a], vy[b] - vy[a], vz[b] - vz[a]};
        double e2[3] = {vx[c] - vx[a], vy[c] - vy[a], vz[c] - vz[a]};
        double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                        e1[0] * e2[1] - e1[1] * e2[0]};
        double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(len > 0.0) || !std::isfinite(len))
            fail(H2B_EINVAL, "triangle " + std::to_string(i) + " has zero area");
        m->area[i] = 0.5 * len;
        m->nx[i] = cr[0] / len;
        m->ny[i] = cr[1] / len;
        m->nz[i] = cr[2] / len;
        m->cx[i] = (vx[a] + vx[b] + vx[c]) / 3.0;
        m->cy[i] = (vy[a] + vy[b] + vy[c]) / 3.0;
        m->cz[i] = (vz[a] + vz[b] + vz[c]) / 3.0;
        deg[a + 1]++;
        deg[b + 1]++;
        deg[c + 1]++;
    }
    for (int64_t v = 0; v < nv; ++v) deg[v + 1] += deg[v];
    m->vt_ptr = deg;
    m->vt_idx.resize(deg[nv]);
    std::vector<int64_t> fill(deg.begin(), deg.end() - 1);
    for (int64_t i = 0; i < nt; ++i) {
        m->vt_idx[fill[t0[i]]++] = (int32_t)i;
        m->vt_idx[fill[t1[i]]++] = (int32_t)i;
        m->vt_idx[fill[t2[i]]++] = (int32_t)i;
    }
    return m;
}

// ---------------------------------------------------------------- trees

double Tree::diam(int c) const
{
    const double *b = &box[6 * (size_t)c];
    double dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return std::sqrt((dx * dx + dy * dy) + dz * dz);
}

double box_dist(const Tree &a, int t, const Tree &b, int s)
{
    const double *p = &a.box[6 * (size_t)t];
    const double *q = &b.box[6 * (size_t)s];
    double g[3];
    for (int d = 0; d < 3; ++d) g[d] = std::max(0.0, std::max(q[d] - p[3 + d], p[d] - q[3 + d]));
    return std::sqrt((g[0] * g[0] + g[1] * g[1]) + g[2] * g[2]);
}

std::shared_ptr<Tree> build_tree(std::shared_ptr<const Mesh> mesh, h2b_space space, int leaf)
{
    if (leaf < 1) fail(H2B_EINVAL, "leaf size must be >= 1");
    if (space != H2B_P0 && space != H2B_P1) fail(H2B_EINVAL, "unknown space");
    auto tr = std::make_shared<Tree>();
    tr->mesh = mesh;
    tr->space = space;
    tr->leaf = leaf;
    const Mesh &m = *mesh;
    const int64_t n = (space == H2B_P0) ? m.nt : m.nv;
    tr->n = n;
    const double *P[3];
    if (space == H2B_P0) {
        P[0] = m.cx.data();
        P[1] = m.cy.data();
        P[2] = m.cz.data();
    } else {
        P[0] = m.vx.data();
        P[1] = m.vy.data();
        P[2] = m.vz.data();
    }
    tr->perm.resize(n);
    std::iota(tr->perm.begin(), tr->perm.end(), 0);
    int32_t *perm = tr->perm.data();

    std::function<int(int32_t, int32_t, int, int)> split = [&](int32_t b, int32_t e, int lev,
                                                               int par) -> int {
        int id = (int)tr->begin.size();
        tr->begin.push_back(b);
        tr->end.push_back(e);
        tr->parent.push_back(par);
        tr->child0.push_back(-1);
        tr->child1.push_back(-1);
        tr->nchild.push_back(0);
        tr->level.push_back(lev);
        if (e - b <= leaf) return id;
        double lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = hi[d] = P[d][perm[b]];
            for (int32_t k = b + 1; k < e; ++k) {
                double v = P[d][perm[k]];
                lo[d] = std::min(lo[d], v);
                hi[d] = std::max(hi[d], v);
            }
        }
        double ext[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        int axes[3] = {0, 1, 2};
        std::stable_sort(axes, axes + 3, [&](int x, int y) { return ext[x] > ext[y]; });
        for (int k = 0; k < 3; ++k) {
            int ax = axes[k];
            double mid = 0.5 * (lo[ax] + hi[ax]);
            const double *pa = P[ax];
            int32_t cnt = 0;
            for (int32_t j = b; j < e; ++j) cnt += (pa[perm[j]] <= mid);
            if (cnt == 0 || cnt == e - b) continue;
            std::stable_partition(perm + b, perm + e, [&](int32_t i) { return pa[i] <= mid; });
            int c0 = split(b, b + cnt, lev + 1, id);
            int c1 = split(b + cnt, e, lev + 1, id);
            tr->child0[id] = c0;
            tr->child1[id] = c1;
            tr->nchild[id] = 2;
            break;
        }
        return id;
    };
    split(0, (int32_t)n, 0, -1);

    const int64_t nc = tr->nclusters();
    tr->box.assign(6 * nc, 0.0);
    // leaf boxes from the supports, parents as unions (children have larger ids)
    for (int64_t c = nc - 1; c >= 0; --c) {
        double *bx = &tr->box[6 * c];
        bx[0] = bx[1] = bx[2] = INFINITY;
        bx[3] = bx[4] = bx[5] = -INFINITY;
        auto add_vertex = [&](int32_t v) {
            double p[3] = {m.vx[v], m.vy[v], m.vz[v]};
            for (int d = 0; d < 3; ++d) {
                bx[d] = std::min(bx[d], p[d]);
                bx[3 + d] = std::max(bx[3 + d], p[d]);
            }
        };
        auto add_triangle = [&](int32_t t) {
            add_vertex(m.t0[t]);
            add_vertex(m.t1[t]);
            add_vertex(m.t2[t]);
        };
        if (tr->nchild[c] == 0) {
            for (int32_t k = tr->begin[c]; k < tr->end[c]; ++k) {
                int32_t i = perm[k];
                if (space == H2B_P0) {
                    add_triangle(i);
                } else {
                    for (int64_t a = m.vt_ptr[i]; a < m.vt_ptr[i + 1]; ++a) add_triangle(m.vt_idx[a]);
                }
            }
        } else {
            int c0 = tr->child0[c], c1 = tr->child1[c];
            for (int cc : {c0, c1}) {
                const double *cb = &tr->box[6 * (size_t)cc];
                for (int d = 0; d < 3; ++d) {
                    bx[d] = std::min(bx[d], cb[d]);
                    bx[3 + d] = std::max(bx[3 + d], cb[3 + d]);
                }
            }
        }
    }
    int maxlev = 0;
    for (int64_t c = 0; c < nc; ++c) {
        maxlev = std::max(maxlev, tr->level[c]);
        if (tr->nchild[c] == 0) tr->leaves.push_back((int32_t)c);
    }
    tr->nlevels = maxlev + 1;
    tr->by_level.assign(tr->nlevels, {});
    for (int64_t c = 0; c < nc; ++c) tr->by_level[tr->level[c]].push_back((int32_t)c);
    return tr;
}

// --------------------------------------------------------------- blocks

std::shared_ptr<Blocks> build_blocks(std::shared_ptr<const Tree> rows,
                                     std::shared_ptr<const Tree> cols, double eta,
                                     bool far_disabled)
{
    if (rows->mesh != cols->mesh) fail(H2B_EINVAL, "row and column trees belong to different meshes");
    if (rows->space != H2B_P0) fail(H2B_EINVAL, "row tree must be a P0 (triangle) tree");
    if (!(eta > 0.0)) fail(H2B_EINVAL, "eta must be positive");
    auto bl = std::make_shared<Blocks>();
    bl->rows = rows;
    bl->cols = cols;
    bl->eta = eta;
    bl->far_disabled = far_disabled;
    const Tree &R = *rows, &C = *cols;
    auto children = [](const Tree &T, int c, int out[2]) {
        out[0] = T.child0[c];
        out[1] = T.child1[c];
    };
    std::function<void(int, int)> rec = [&](int t, int s) {
        if (!far_disabled) {
            double dt = R.diam(t), ds = C.diam(s);
            if (std::max(dt, ds) <= 2.0 * eta * box_dist(R, t, C, s)) {
                bl->far_t.push_back(t);
                bl->far_s.push_back(s);
                return;
            }
        }
        bool lt = R.nchild[t] == 0, ls = C.nchild[s] == 0;
        if (lt && ls) {
            bl->near_t.push_back(t);
            bl->near_s.push_back(s);
        } else if (lt) {
            int ch[2];
            children(C, s, ch);
            rec(t, ch[0]);
            rec(t, ch[1]);
        } else if (ls) {
            int ch[2];
            children(R, t, ch);
            rec(ch[0], s);
            rec(ch[1], s);
        } else {
            int ct[2], cs[2];
            children(R, t, ct);
            children(C, s, cs);
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) rec(ct[a], cs[b]);
        }
    };
    rec(0, 0);
    return bl;
}

// ------------------------------------------------------------ numerics

void sym_eig(int n, std::vector<double> &a, std::vector<double> &ev, std::vector<double> &z)
{
    z.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) z[(size_t)i * n + i] = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i) {
            diag += a[(size_t)i * n + i] * a[(size_t)i * n + i];
            for (int j = i + 1; j < n; ++j) off += a[(size_t)i * n + j] * a[(size_t)i * n + j];
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = a[(size_t)p * n + p], aqq = a[(size_t)q * n + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = a[(size_t)k * n + p], akq = a[(size_t)k * n + q];
                    a[(size_t)k * n + p] = c * akp - s * akq;
                    a[(size_t)k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a[(size_t)p * n + k], aqk = a[(size_t)q * n + k];
                    a[(size_t)p * n + k] = c * apk - s * aqk;
                    a[(size_t)q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double zkp = z[(size_t)k * n + p], zkq = z[(size_t)k * n + q];
                    z[(size_t)k * n + p] = c * zkp - s * zkq;
                    z[(size_t)k * n + q] = s * zkp + c * zkq;
                }
            }
    }
    // sort descending
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        return a[(size_t)x * n + x] > a[(size_t)y * n + y];
    });
    ev.resize(n);
    std::vector<double> zs((size_t)n * n);
    for (int j = 0; j < n; ++j) {
        ev[j] = a[(size_t)idx[j] * n + idx[j]];
        for (int k = 0; k < n; ++k) zs[(size_t)k * n + j] = z[(size_t)k * n + idx[j]];
    }
    z.swap(zs);
}

void gauss_legendre_unit(int q, std::vector<double> &t, std::vector<double> &w)
{
    // Golub-Welsch on [-1,1]: Jacobi matrix with zero diagonal and off-diagonal
    // k / sqrt(4k^2 - 1); nodes = eigenvalues, weights = 2 v_0^2.
    std::vector<double> J((size_t)q * q, 0.0), ev, z;
    for (int k = 1; k < q; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        J[(size_t)(k - 1) * q + k] = b;
        J[(size_t)k * q + k - 1] = b;
    }
    sym_eig(q, J, ev, z);
    t.resize(q);
    w.resize(q);
    // ev is descending; map to ascending nodes on [0,1]
    for (int i = 0; i < q; ++i) {
        int j = q - 1 - i;
        double x = ev[j];
        // one Newton step on P_q for full accuracy of the node
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= q; ++k) {
            double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        double dp = (q == 1) ? 1.0 : q * (x * p1 - p0) / (x * x - 1.0);
        x -= p1 / dp;
        t[i] = 0.5 * (x + 1.0);
        w[i] = z[(size_t)0 * q + j] * z[(size_t)0 * q + j];  // 2 v0^2 on [-1,1] -> v0^2 on [0,1]
    }
}

void cheb_axes(const Tree &tr, int c, int m, double *pts)
{
    const double *b = &tr.box[6 * (size_t)c];
    double d = tr.diam(c);
    for (int ax = 0; ax < 3; ++ax) {
        double lo = b[ax], hi = b[3 + ax];
        if (hi - lo < 1e-12 * d) {
            double mid = 0.5 * (lo + hi);
            lo = mid - 0.5e-12 * d;
            hi = mid + 0.5e-12 * d;
        }
        for (int i = 0; i < m; ++i)
            pts[ax * m + i] = 0.5 * (lo + hi) + 0.5 * (hi - lo) * std::cos(M_PI * (2 * i + 1) / (2 * m));
    }
}

}  // namespace h2b
