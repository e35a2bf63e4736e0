/*
 * bem_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU reference for the Galerkin matrices of
 * the 3-D Laplace boundary integral operators.  Nothing in the product path
 * may link or call this file; only the tests, the smoke check and the CPU
 * baseline of the benchmark do.  It shares no source with the HIP library.
 *
 * What it computes (paper, Section 1, eqs. (slp) and (dlp)):
 *   g(x,y)      = 1 / (4 pi |x-y|)                      (Section 1, kernel g)
 *   dg/dn_y     = <x-y, n_y> / (4 pi |x-y|^3)           (normal derivative of g)
 *   G_ij        = int_{tau_i} int_{tau_j} g(x,y) dy dx  (psi_i = indicator of triangle i)
 *   K_ij        = int_{tau_i} int_Gamma dg/dn_y(x,y) phi_j(y) dy dx
 *                 (phi_j = continuous piecewise linear nodal function of vertex j;
 *                  Section 5 fixes these two discrete spaces)
 *
 * Every entry is computed by four-dimensional Gauss-Legendre quadrature of the
 * pair of flat triangles.  Pairs that touch (same triangle, common edge, common
 * vertex) use Sauter-Schwab regularising substitutions, the singular quadrature
 * that Section 5 prescribes for the near field; disjoint pairs use the tensor
 * product of collapsed (Duffy) Gauss rules on each triangle.  q points per
 * dimension throughout ("q_near" of Table 1).
 *
 * Reference triangle  T = {(u1,u2) : 0 <= u2 <= u1 <= 1}, mapped to a flat
 * triangle with ordered corners (P0,P1,P2) by
 *   chi(u1,u2) = P0 + u1 (P1-P0) + u2 (P2-P1),  |det| = 2 |tau|,
 * so the barycentric weights of P0,P1,P2 at chi(u) are (1-u1, u1-u2, u2).
 *
 * Ordering of a touching pair: the shared corners come first in both triangles
 * (for a common edge, the two shared vertices in increasing global index; for a
 * common vertex, the shared one followed by the remaining corners in the
 * triangle's own cyclic order).  Identical and disjoint pairs keep the stored
 * order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_QMAX 32

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ---------------------------------------------------------------- threads */

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------ Gauss-Legendre */

/* Nodes and weights of the q-point Gauss-Legendre rule on [0,1], ascending.
 * Nodes are the roots of the Legendre polynomial P_q, found by Newton's method
 * with P_q and P_q' from the three-term recurrence
 *   k P_k(z) = (2k-1) z P_{k-1}(z) - (k-1) P_{k-2}(z),
 *   P_q'(z)  = q (z P_q(z) - P_{q-1}(z)) / (z^2 - 1),
 * and weights 2 / ((1-z^2) P_q'(z)^2) on [-1,1] (halved for [0,1]). */
int orc_gauss_legendre01(int q, double *t, double *w)
{
    if (q < 1 || q > ORC_QMAX) return -1;
    for (int i = 0; i < q; ++i) {
        double z = cos(ORC_PI * (i + 0.75) / (q + 0.5));
        double pq = 0.0, pqm1 = 0.0, dp = 1.0;
        for (int it = 0; it < 200; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            pq = p1;
            pqm1 = p0;
            dp = (q == 1) ? 1.0 : q * (z * pq - pqm1) / (z * z - 1.0);
            double dz = pq / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        /* derivative at the converged root */
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = (q == 1) ? 1.0 : q * (z * p1 - p0) / (z * z - 1.0);
        }
        /* z runs from near +1 downwards, so (1 - z)/2 ascends */
        t[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------ geometry */

static void sub3(const double *a, const double *b, double *c)
{
    c[0] = a[0] - b[0];
    c[1] = a[1] - b[1];
    c[2] = a[2] - b[2];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Outward unit normal and area of triangle (a,b,c) in stored (counter-clockwise
 * seen from outside) order. */
static double tri_normal(const double *a, const double *b, const double *c, double *n)
{
    double e1[3], e2[3], cr[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, cr);
    double len = sqrt(dot3(cr, cr));
    n[0] = cr[0] / len;
    n[1] = cr[1] / len;
    n[2] = cr[2] / len;
    return 0.5 * len;
}

/* ------------------------------------------- pair relation and ordering */

/* Number of shared vertices (3 identical, 2 edge, 1 vertex, 0 disjoint) and the
 * corner order of both triangles used by the quadrature (slots into the stored
 * vertex triples). */
static int pair_order(const int32_t *ti, const int32_t *tj, int pi[3], int pj[3])
{
    int si[3], sj[3], ns = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ti[a] == tj[b]) {
                si[ns] = a;
                sj[ns] = b;
                ++ns;
            }
    if (ns == 3 || ns == 0) {
        for (int a = 0; a < 3; ++a) pi[a] = pj[a] = a;
        return ns;
    }
    if (ns == 2) {
        /* shared vertices in increasing global index, then the free corner */
        int lo = 0, hi = 1;
        if (ti[si[1]] < ti[si[0]]) {
            lo = 1;
            hi = 0;
        }
        pi[0] = si[lo];
        pi[1] = si[hi];
        pi[2] = 3 - si[0] - si[1];
        pj[0] = sj[lo];
        pj[1] = sj[hi];
        pj[2] = 3 - sj[0] - sj[1];
        return 2;
    }
    /* one shared vertex, then the triangle's own cyclic order */
    for (int a = 0; a < 3; ++a) {
        pi[a] = (si[0] + a) % 3;
        pj[a] = (sj[0] + a) % 3;
    }
    return 1;
}

/* ----------------------------------------- Sauter-Schwab substitutions */

/* For a touching pair with relation rel (3, 2, 1) and sub-region r, map the
 * unit-cube point (s,e1,e2,e3) to reference points x = (x1,x2), y = (y1,y2) in
 * T x T and return the Jacobian of the substitution.  The sub-regions of each
 * relation tile T x T exactly; the Jacobians vanish where x = y so that a
 * 1/|x-y| or 1/|x-y|^2 singularity becomes bounded.
 *   identical  : 6 regions, Jacobian s^3 e1^2 e2
 *   common edge: 5 regions (shared edge u2 = 0), Jacobians s^3 e1^2 and s^3 e1^2 e2
 *   common vertex: 2 regions (shared corner u = 0), Jacobian s^3 e2 */
static double ss_map(int rel, int r, double s, double e1, double e2, double e3,
                     double *x, double *y)
{
    if (rel == 3) {
        double jac = s * s * s * e1 * e1 * e2;
        switch (r) {
        case 0:
            x[0] = s; x[1] = s * (1.0 - e1 + e1 * e2);
            y[0] = s * (1.0 - e1 * e2 * e3); y[1] = s * (1.0 - e1);
            break;
        case 1:
            x[0] = s * (1.0 - e1 * e2 * e3); x[1] = s * (1.0 - e1);
            y[0] = s; y[1] = s * (1.0 - e1 + e1 * e2);
            break;
        case 2:
            x[0] = s; x[1] = s * e1 * (1.0 - e2 + e2 * e3);
            y[0] = s * (1.0 - e1 * e2); y[1] = s * e1 * (1.0 - e2);
            break;
        case 3:
            x[0] = s * (1.0 - e1 * e2); x[1] = s * e1 * (1.0 - e2);
            y[0] = s; y[1] = s * e1 * (1.0 - e2 + e2 * e3);
            break;
        case 4:
            x[0] = s * (1.0 - e1 * e2 * e3); x[1] = s * e1 * (1.0 - e2 * e3);
            y[0] = s; y[1] = s * e1 * (1.0 - e2);
            break;
        default:
            x[0] = s; x[1] = s * e1 * (1.0 - e2);
            y[0] = s * (1.0 - e1 * e2 * e3); y[1] = s * e1 * (1.0 - e2 * e3);
            break;
        }
        return jac;
    }
    if (rel == 2) {
        double jac = s * s * s * e1 * e1;
        switch (r) {
        case 0:
            x[0] = s; x[1] = s * e1 * e3;
            y[0] = s * (1.0 - e1 * e2); y[1] = s * e1 * (1.0 - e2);
            return jac;
        case 1:
            x[0] = s; x[1] = s * e1;
            y[0] = s * (1.0 - e1 * e2 * e3); y[1] = s * e1 * e2 * (1.0 - e3);
            return jac * e2;
        case 2:
            x[0] = s * (1.0 - e1 * e2); x[1] = s * e1 * (1.0 - e2);
            y[0] = s; y[1] = s * e1 * e2 * e3;
            return jac * e2;
        case 3:
            x[0] = s * (1.0 - e1 * e2 * e3); x[1] = s * e1 * e2 * (1.0 - e3);
            y[0] = s; y[1] = s * e1;
            return jac * e2;
        default:
            x[0] = s * (1.0 - e1 * e2 * e3); x[1] = s * e1 * (1.0 - e2 * e3);
            y[0] = s; y[1] = s * e1 * e2;
            return jac * e2;
        }
    }
    /* rel == 1 */
    if (r == 0) {
        x[0] = s; x[1] = s * e1;
        y[0] = s * e2; y[1] = s * e2 * e3;
    } else {
        x[0] = s * e2; x[1] = s * e2 * e3;
        y[0] = s; y[1] = s * e1;
    }
    return s * s * s * e2;
}

static void chi(const double P[3][3], const double *u, double *p)
{
    for (int d = 0; d < 3; ++d)
        p[d] = P[0][d] + u[0] * (P[1][d] - P[0][d]) + u[1] * (P[2][d] - P[1][d]);
}

/* Galerkin integral of one triangle pair.
 *   dlp = 0: out[0] = int_X int_Y g(x,y) dy dx
 *   dlp = 1: out[c] = int_X int_Y dg/dn_y(x,y) lambda_c(y) dy dx, c = corner of Y
 *            in the given order, ny = unit normal of Y.
 * X and Y hold the corners in quadrature order (see pair_order). */
static void pair_integral(int dlp, const double X[3][3], const double Y[3][3],
                          const double *ny, int rel, int q, const double *t,
                          const double *w, double *out)
{
    double ex[3], ey[3], cr[3];
    sub3(X[1], X[0], ex);
    sub3(X[2], X[1], ey);
    cross3(ex, ey, cr);
    double jx = sqrt(dot3(cr, cr));
    sub3(Y[1], Y[0], ex);
    sub3(Y[2], Y[1], ey);
    cross3(ex, ey, cr);
    double jy = sqrt(dot3(cr, cr));

    int nreg = (rel == 3) ? 6 : (rel == 2) ? 5 : (rel == 1) ? 2 : 1;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (int r = 0; r < nreg; ++r)
        for (int a = 0; a < q; ++a)
            for (int b = 0; b < q; ++b)
                for (int c = 0; c < q; ++c)
                    for (int d = 0; d < q; ++d) {
                        double xh[2], yh[2], jac;
                        if (rel == 0) {
                            /* collapsed Gauss rule on each triangle */
                            xh[0] = t[a]; xh[1] = t[a] * t[b];
                            yh[0] = t[c]; yh[1] = t[c] * t[d];
                            jac = t[a] * t[c];
                        } else {
                            jac = ss_map(rel, r, t[a], t[b], t[c], t[d], xh, yh);
                        }
                        double wt = jac * w[a] * w[b] * w[c] * w[d];
                        double px[3], py[3], dv[3];
                        chi(X, xh, px);
                        chi(Y, yh, py);
                        sub3(px, py, dv);
                        double r2 = dot3(dv, dv);
                        double rr = sqrt(r2);
                        if (!dlp) {
                            acc0 += wt / rr;
                        } else {
                            double kv = wt * dot3(dv, ny) / (r2 * rr);
                            acc0 += kv * (1.0 - yh[0]);
                            acc1 += kv * (yh[0] - yh[1]);
                            acc2 += kv * yh[1];
                        }
                    }
    double scale = jx * jy / (4.0 * ORC_PI);
    out[0] = acc0 * scale;
    out[1] = acc1 * scale;
    out[2] = acc2 * scale;
}

/* ------------------------------------------------------------- entries */

typedef struct {
    const double *V;   /* vertices, xyz interleaved, nv x 3 */
    const int32_t *T;  /* triangles, nt x 3, counter-clockwise seen from outside */
    int64_t nv, nt;
    int q;
    double t[ORC_QMAX], w[ORC_QMAX];
} orc_mesh;

static int mesh_init(orc_mesh *m, int64_t nv, const double *V, int64_t nt,
                     const int32_t *T, int q)
{
    m->V = V;
    m->T = T;
    m->nv = nv;
    m->nt = nt;
    m->q = q;
    return orc_gauss_legendre01(q, m->t, m->w);
}

/* G_ij, triangle i carrying x and triangle j carrying y. */
static double slp_entry(const orc_mesh *m, int64_t i, int64_t j)
{
    const int32_t *ti = m->T + 3 * i, *tj = m->T + 3 * j;
    int pi[3], pj[3];
    int rel = pair_order(ti, tj, pi, pj);
    double X[3][3], Y[3][3], out[3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
            X[a][d] = m->V[3 * ti[pi[a]] + d];
            Y[a][d] = m->V[3 * tj[pj[a]] + d];
        }
    pair_integral(0, X, Y, NULL, rel, m->q, m->t, m->w, out);
    return out[0];
}

/* Contributions of triangle pair (tau_i, tau_j) to K: val[c] belongs to column
 * T[j][c] (stored corner c of triangle j). */
static void dlp_pair(const orc_mesh *m, int64_t i, int64_t j, double val[3])
{
    const int32_t *ti = m->T + 3 * i, *tj = m->T + 3 * j;
    int pi[3], pj[3];
    int rel = pair_order(ti, tj, pi, pj);
    double X[3][3], Y[3][3], out[3], ny[3];
    for (int a = 0; a < 3; ++a)
        for (int d = 0; d < 3; ++d) {
            X[a][d] = m->V[3 * ti[pi[a]] + d];
            Y[a][d] = m->V[3 * tj[pj[a]] + d];
        }
    tri_normal(m->V + 3 * tj[0], m->V + 3 * tj[1], m->V + 3 * tj[2], ny);
    pair_integral(1, X, Y, ny, rel, m->q, m->t, m->w, out);
    for (int a = 0; a < 3; ++a) val[pj[a]] = out[a];
}

/* ----------------------------------------------------------- public API */

/* Dense G (nt x nt, row-major). */
int orc_slp_dense(int64_t nv, const double *V, int64_t nt, const int32_t *T,
                  int q, double *G)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nt; ++i)
        for (int64_t j = 0; j < nt; ++j) G[i * nt + j] = slp_entry(&m, i, j);
    return 0;
}

/* Dense K (nt x nv, row-major). */
int orc_dlp_dense(int64_t nv, const double *V, int64_t nt, const int32_t *T,
                  int q, double *K)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nt; ++i) {
        double *row = K + i * nv;
        for (int64_t c = 0; c < nv; ++c) row[c] = 0.0;
        for (int64_t j = 0; j < nt; ++j) {
            double val[3];
            dlp_pair(&m, i, j, val);
            for (int c = 0; c < 3; ++c) row[T[3 * j + c]] += val[c];
        }
    }
    return 0;
}

/* Selected rows of G x (trans = 0) or G^T x (trans = 1):
 *   y[r] = sum_j G[rows[r], j] x[j]      or      y[r] = sum_i G[i, rows[r]] x[i]. */
int orc_slp_rows(int64_t nv, const double *V, int64_t nt, const int32_t *T, int q,
                 int trans, int64_t nrows, const int64_t *rows, const double *x,
                 double *y)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t k = rows[r];
        double s = 0.0;
        for (int64_t j = 0; j < nt; ++j)
            s += (trans ? slp_entry(&m, j, k) : slp_entry(&m, k, j)) * x[j];
        y[r] = s;
    }
    return 0;
}

/* Selected rows of K x (trans = 0: rows are triangles, x has nv entries) or of
 * K^T x (trans = 1: rows are vertices, x has nt entries).
 *   (K x)_i   = int_{tau_i} int_Gamma dg/dn_y(x,y) u(y) dy dx,  u = sum_j x_j phi_j
 *   (K^T x)_j = sum_i x_i K_ij,  K_ij summed over the triangles around vertex j. */
int orc_dlp_rows(int64_t nv, const double *V, int64_t nt, const int32_t *T, int q,
                 int trans, int64_t nrows, const int64_t *rows, const double *x,
                 double *y)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t k = rows[r];
        double s = 0.0;
        if (!trans) {
            for (int64_t j = 0; j < nt; ++j) {
                double val[3];
                dlp_pair(&m, k, j, val);
                for (int c = 0; c < 3; ++c) s += val[c] * x[T[3 * j + c]];
            }
        } else {
            for (int64_t j = 0; j < nt; ++j) {
                int c = -1;
                for (int a = 0; a < 3; ++a)
                    if (T[3 * j + a] == k) c = a;
                if (c < 0) continue;
                for (int64_t i = 0; i < nt; ++i) {
                    double val[3];
                    dlp_pair(&m, i, j, val);
                    s += val[c] * x[i];
                }
            }
        }
        y[r] = s;
    }
    return 0;
}

/* Single entries, for pinning individual quadrature cases. */
double orc_slp_entry(int64_t nv, const double *V, int64_t nt, const int32_t *T,
                     int q, int64_t i, int64_t j)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return NAN;
    if (i < 0 || j < 0 || i >= nt || j >= nt) return NAN;
    return slp_entry(&m, i, j);
}

int orc_dlp_pair(int64_t nv, const double *V, int64_t nt, const int32_t *T, int q,
                 int64_t i, int64_t j, double *val)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
    if (i < 0 || j < 0 || i >= nt || j >= nt) return -1;
    dlp_pair(&m, i, j, val);
    return 0;
}

/* Entries of the dense matrices at given rows and columns (row-major
 * nr x nc): out[a][b] = G[rows[a], cols[b]] (cols are triangles), or
 * K[rows[a], cols[b]] (cols are vertices; K_ij sums the slot of vertex j over
 * the pairs (i, tau) of the triangles tau around j, in increasing order of
 * tau, as the dense K does). */
int orc_slp_block(int64_t nv, const double *V, int64_t nt, const int32_t *T, int q,
                  int64_t nr, const int64_t *rows, int64_t nc, const int64_t *cols,
                  double *out)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
    for (int64_t a = 0; a < nr; ++a)
        if (rows[a] < 0 || rows[a] >= nt) return -1;
    for (int64_t b = 0; b < nc; ++b)
        if (cols[b] < 0 || cols[b] >= nt) return -1;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t a = 0; a < nr; ++a)
        for (int64_t b = 0; b < nc; ++b)
            out[a * nc + b] = slp_entry(&m, rows[a], cols[b]);
    return 0;
}

int orc_dlp_block(int64_t nv, const double *V, int64_t nt, const int32_t *T, int q,
                  int64_t nr, const int64_t *rows, int64_t nc, const int64_t *cols,
                  double *out)
{
    orc_mesh m;
    if (mesh_init(&m, nv, V, nt, T, q)) return -1;
    for (int64_t a = 0; a < nr; ++a)
        if (rows[a] < 0 || rows[a] >= nt) return -1;
    for (int64_t b = 0; b < nc; ++b)
        if (cols[b] < 0 || cols[b] >= nv) return -1;
    /* triangles around each vertex, in increasing triangle order */
    int64_t *ptr = calloc((size_t)nv + 1, sizeof(int64_t));
    int64_t *adj = malloc(sizeof(int64_t) * (size_t)(3 * nt));
    if (!ptr || !adj) {
        free(ptr);
        free(adj);
        return -2;
    }
    for (int64_t j = 0; j < 3 * nt; ++j) ptr[T[j] + 1]++;
    for (int64_t v = 0; v < nv; ++v) ptr[v + 1] += ptr[v];
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)nv);
    if (!fill) {
        free(ptr);
        free(adj);
        return -2;
    }
    for (int64_t v = 0; v < nv; ++v) fill[v] = ptr[v];
    for (int64_t j = 0; j < nt; ++j)
        for (int c = 0; c < 3; ++c) adj[fill[T[3 * j + c]]++] = j;
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t a = 0; a < nr; ++a)
        for (int64_t b = 0; b < nc; ++b) {
            const int64_t vtx = cols[b];
            double s = 0.0;
            for (int64_t e = ptr[vtx]; e < ptr[vtx + 1]; ++e) {
                const int64_t tau = adj[e];
                double val[3];
                dlp_pair(&m, rows[a], tau, val);
                for (int c = 0; c < 3; ++c)
                    if (T[3 * tau + c] == vtx) s += val[c];
            }
            out[a * nc + b] = s;
        }
    free(fill);
    free(ptr);
    free(adj);
    return 0;
}
