// HIP kernels for gfx950: nearfield quadrature, interpolation bases, transfer
// and coupling matrices, and the panel products that make up the H^2
// matrix-vector product.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"

namespace h2b {

namespace {

constexpr double INV_4PI = 0.0795774715459476678844418816862571810;  // 1 / (4 pi)
constexpr int NT = 256;                                             // threads per workgroup

inline int blocks_for(int64_t n, int per = NT)
{
    int64_t b = (n + per - 1) / per;
    return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 1 << 20);
}

// ===================================================================
//  Triangle-pair quadrature (paper, Section 5: Sauter-Schwab-Erichsen)
// ===================================================================
//
// A flat triangle with ordered corners (P0,P1,P2) is parametrised over the
// reference triangle {0 <= u2 <= u1 <= 1} by P0 + u1 (P1-P0) + u2 (P2-P1).
// For a touching pair both triangles start at the shared corner, so every
// Sauter-Schwab substitution has the form x = xi X(eta), y = xi Y(eta) in
// reference coordinates with Jacobian xi^3 J(eta), and the physical difference
// is x - y = xi D(eta).  The integrands of G and K are then polynomials of
// degree <= 2 in xi divided by |D|, so the xi-direction of the tensor Gauss
// rule is exact and is summed in closed form; the remaining three directions
// use the q-point Gauss rule per dimension.

struct Tri {
    double p[3];   // first corner
    double e1[3];  // P1 - P0
    double e2[3];  // P2 - P1
};

__device__ inline void load_tri(const GeoDev &g, int c0, int c1, int c2, Tri &T)
{
    double a[3] = {g.vx[c0], g.vy[c0], g.vz[c0]};
    double b[3] = {g.vx[c1], g.vy[c1], g.vz[c1]};
    double c[3] = {g.vx[c2], g.vy[c2], g.vz[c2]};
    for (int d = 0; d < 3; ++d) {
        T.p[d] = a[d];
        T.e1[d] = b[d] - a[d];
        T.e2[d] = c[d] - b[d];
    }
}

__device__ inline double tri_jac(const Tri &T)
{
    double c0 = T.e1[1] * T.e2[2] - T.e1[2] * T.e2[1];
    double c1 = T.e1[2] * T.e2[0] - T.e1[0] * T.e2[2];
    double c2 = T.e1[0] * T.e2[1] - T.e1[1] * T.e2[0];
    return sqrt(c0 * c0 + c1 * c1 + c2 * c2);
}

// Reference directions X(eta), Y(eta) and J(eta) of region r of the relation
// with ns shared vertices (3: six regions, 2: five regions, 1: two regions).
__device__ inline double ss_dirs(int ns, int r, double a, double b, double c, double X[2],
                                 double Y[2])
{
    const double ab = a * b, abc = a * b * c;
    if (ns == 3) {
        switch (r) {
        case 0: X[0] = 1.0; X[1] = 1.0 - a + ab; Y[0] = 1.0 - abc; Y[1] = 1.0 - a; break;
        case 1: X[0] = 1.0 - abc; X[1] = 1.0 - a; Y[0] = 1.0; Y[1] = 1.0 - a + ab; break;
        case 2: X[0] = 1.0; X[1] = a * (1.0 - b + b * c); Y[0] = 1.0 - ab; Y[1] = a * (1.0 - b); break;
        case 3: X[0] = 1.0 - ab; X[1] = a * (1.0 - b); Y[0] = 1.0; Y[1] = a * (1.0 - b + b * c); break;
        case 4: X[0] = 1.0 - abc; X[1] = a * (1.0 - b * c); Y[0] = 1.0; Y[1] = a * (1.0 - b); break;
        default: X[0] = 1.0; X[1] = a * (1.0 - b); Y[0] = 1.0 - abc; Y[1] = a * (1.0 - b * c); break;
        }
        return a * a * b;
    }
    if (ns == 2) {
        switch (r) {
        case 0: X[0] = 1.0; X[1] = a * c; Y[0] = 1.0 - ab; Y[1] = a * (1.0 - b); return a * a;
        case 1: X[0] = 1.0; X[1] = a; Y[0] = 1.0 - abc; Y[1] = ab * (1.0 - c); break;
        case 2: X[0] = 1.0 - ab; X[1] = a * (1.0 - b); Y[0] = 1.0; Y[1] = abc; break;
        case 3: X[0] = 1.0 - abc; X[1] = ab * (1.0 - c); Y[0] = 1.0; Y[1] = a; break;
        default: X[0] = 1.0 - abc; X[1] = a * (1.0 - b * c); Y[0] = 1.0; Y[1] = ab; break;
        }
        return a * a * b;
    }
    if (r == 0) {
        X[0] = 1.0; X[1] = a; Y[0] = b; Y[1] = b * c;
    } else {
        X[0] = b; X[1] = b * c; Y[0] = 1.0; Y[1] = a;
    }
    return b;
}

// Corner order of a pair: returns the number of shared vertices; ox/oy are the
// stored corner slots in quadrature order (shared corners first: a common edge
// in increasing global vertex index, a common vertex followed by the rest in
// the triangle's cyclic order).
__device__ inline int pair_slots(const int vx[3], const int vy[3], int ox[3], int oy[3])
{
    int ns = 0, sx[3], sy[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            if (vx[a] == vy[b]) {
                sx[ns] = a;
                sy[ns] = b;
                ++ns;
            }
    if (ns == 2) {
        int f = (vx[sx[0]] < vx[sx[1]]) ? 0 : 1;
        ox[0] = sx[f]; ox[1] = sx[1 - f]; ox[2] = 3 - sx[0] - sx[1];
        oy[0] = sy[f]; oy[1] = sy[1 - f]; oy[2] = 3 - sy[0] - sy[1];
    } else if (ns == 1) {
        for (int a = 0; a < 3; ++a) {
            ox[a] = (sx[0] + a) % 3;
            oy[a] = (sy[0] + a) % 3;
        }
    } else {
        for (int a = 0; a < 3; ++a) ox[a] = oy[a] = a;
    }
    return ns;
}

// int_X int_Y g(x,y) dy dx for a touching pair (ns >= 1).
__device__ double slp_touching(int ns, const Tri &X, const Tri &Y, const QuadDev &Q)
{
    const int nreg = (ns == 3) ? 6 : (ns == 2) ? 5 : 2;
    double acc = 0.0;
    for (int r = 0; r < nreg; ++r)
        for (int i = 0; i < Q.q; ++i)
            for (int j = 0; j < Q.q; ++j) {
                const double wij = Q.w[i] * Q.w[j];
                for (int k = 0; k < Q.q; ++k) {
                    double xd[2], yd[2];
                    double jac = ss_dirs(ns, r, Q.t[i], Q.t[j], Q.t[k], xd, yd);
                    double D0 = xd[0] * X.e1[0] + xd[1] * X.e2[0] - yd[0] * Y.e1[0] - yd[1] * Y.e2[0];
                    double D1 = xd[0] * X.e1[1] + xd[1] * X.e2[1] - yd[0] * Y.e1[1] - yd[1] * Y.e2[1];
                    double D2 = xd[0] * X.e1[2] + xd[1] * X.e2[2] - yd[0] * Y.e1[2] - yd[1] * Y.e2[2];
                    acc += wij * Q.w[k] * jac * rsqrt(D0 * D0 + D1 * D1 + D2 * D2);
                }
            }
    // xi^3 / xi integrated over [0,1]
    return acc * (1.0 / 3.0);
}

// int_X int_Y dg/dn_y(x,y) lambda_c(y) dy dx for a touching pair, c = corner of
// Y in quadrature order; ny = unit normal of Y.
__device__ double dlp_touching(int ns, const Tri &X, const Tri &Y, const double ny[3], int c,
                               const QuadDev &Q)
{
    if (ns == 3) return 0.0;  // x - y lies in the plane of the triangle
    const int nreg = (ns == 2) ? 5 : 2;
    double acc = 0.0;
    for (int r = 0; r < nreg; ++r)
        for (int i = 0; i < Q.q; ++i)
            for (int j = 0; j < Q.q; ++j) {
                const double wij = Q.w[i] * Q.w[j];
                for (int k = 0; k < Q.q; ++k) {
                    double xd[2], yd[2];
                    double jac = ss_dirs(ns, r, Q.t[i], Q.t[j], Q.t[k], xd, yd);
                    double D0 = xd[0] * X.e1[0] + xd[1] * X.e2[0] - yd[0] * Y.e1[0] - yd[1] * Y.e2[0];
                    double D1 = xd[0] * X.e1[1] + xd[1] * X.e2[1] - yd[0] * Y.e1[1] - yd[1] * Y.e2[1];
                    double D2 = xd[0] * X.e1[2] + xd[1] * X.e2[2] - yd[0] * Y.e1[2] - yd[1] * Y.e2[2];
                    double ir = rsqrt(D0 * D0 + D1 * D1 + D2 * D2);
                    double kern = (D0 * ny[0] + D1 * ny[1] + D2 * ny[2]) * ir * ir * ir;
                    // barycentric weight of corner c at y = xi Y, integrated against xi
                    double lam = (c == 0) ? (0.5 - yd[0] * (1.0 / 3.0))
                               : (c == 1) ? (yd[0] - yd[1]) * (1.0 / 3.0)
                                          : yd[1] * (1.0 / 3.0);
                    acc += wij * Q.w[k] * jac * kern * lam;
                }
            }
    return acc;
}

// Disjoint pair: collapsed Gauss rule on each triangle (q^2 points each).
// c < 0: single layer; c in 0..2: double layer with barycentric weight of
// corner c of Y.
__device__ double pair_regular(const Tri &X, const Tri &Y, const double ny[3], int c,
                               const QuadDev &Q)
{
    double acc = 0.0;
    for (int i = 0; i < Q.q; ++i) {
        const double u = Q.t[i];
        for (int j = 0; j < Q.q; ++j) {
            const double v = u * Q.t[j];
            const double wx = Q.w[i] * Q.w[j] * u;
            const double x0 = X.p[0] + u * X.e1[0] + v * X.e2[0];
            const double x1 = X.p[1] + u * X.e1[1] + v * X.e2[1];
            const double x2 = X.p[2] + u * X.e1[2] + v * X.e2[2];
            double inner = 0.0;
            for (int k = 0; k < Q.q; ++k) {
                const double s = Q.t[k];
                const double ws = Q.w[k] * s;
                for (int l = 0; l < Q.q; ++l) {
                    const double sv = s * Q.t[l];
                    const double d0 = x0 - (Y.p[0] + s * Y.e1[0] + sv * Y.e2[0]);
                    const double d1 = x1 - (Y.p[1] + s * Y.e1[1] + sv * Y.e2[1]);
                    const double d2 = x2 - (Y.p[2] + s * Y.e1[2] + sv * Y.e2[2]);
                    const double ir = rsqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    double f;
                    if (c < 0) {
                        f = ir;
                    } else {
                        const double lam = (c == 0) ? 1.0 - s : (c == 1) ? s - sv : sv;
                        f = (d0 * ny[0] + d1 * ny[1] + d2 * ny[2]) * ir * ir * ir * lam;
                    }
                    inner += ws * Q.w[l] * f;
                }
            }
            acc += wx * inner;
        }
    }
    return acc;
}

__device__ double slp_entry(const GeoDev &g, int i, int j, const QuadDev &Q)
{
    int vi[3] = {g.t0[i], g.t1[i], g.t2[i]};
    int vj[3] = {g.t0[j], g.t1[j], g.t2[j]};
    int oi[3], oj[3];
    int ns = pair_slots(vi, vj, oi, oj);
    Tri X, Y;
    load_tri(g, vi[oi[0]], vi[oi[1]], vi[oi[2]], X);
    load_tri(g, vj[oj[0]], vj[oj[1]], vj[oj[2]], Y);
    double jj = tri_jac(X) * tri_jac(Y) * INV_4PI;
    double nn[3] = {0, 0, 0};
    double v = (ns == 0) ? pair_regular(X, Y, nn, -1, Q) : slp_touching(ns, X, Y, Q);
    return v * jj;
}

// Contribution of triangle tj to K_{i, vertex} where vertex sits in stored slot
// `slot` of tj.
__device__ double dlp_part(const GeoDev &g, int i, int tj, int slot, const QuadDev &Q)
{
    int vi[3] = {g.t0[i], g.t1[i], g.t2[i]};
    int vj[3] = {g.t0[tj], g.t1[tj], g.t2[tj]};
    int oi[3], oj[3];
    int ns = pair_slots(vi, vj, oi, oj);
    int c = (oj[0] == slot) ? 0 : (oj[1] == slot) ? 1 : 2;
    Tri X, Y;
    load_tri(g, vi[oi[0]], vi[oi[1]], vi[oi[2]], X);
    load_tri(g, vj[oj[0]], vj[oj[1]], vj[oj[2]], Y);
    double ny[3] = {g.nx[tj], g.ny[tj], g.nz[tj]};
    double jj = tri_jac(X) * tri_jac(Y) * INV_4PI;
    double v = (ns == 0) ? pair_regular(X, Y, ny, c, Q) : dlp_touching(ns, X, Y, ny, c, Q);
    return v * jj;
}

// The double-layer integrals of a pair for all three barycentric weights of
// Y at once (corners in quadrature order): the same rules as dlp_touching and
// pair_regular, sharing every kernel evaluation among the three corners.
__device__ void dlp_touching3(int ns, const Tri &X, const Tri &Y, const double ny[3], const QuadDev &Q,
                              double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    if (ns == 3) return;  // x - y lies in the plane of the triangle
    const int nreg = (ns == 2) ? 5 : 2;
    for (int r = 0; r < nreg; ++r)
        for (int i = 0; i < Q.q; ++i)
            for (int j = 0; j < Q.q; ++j) {
                const double wij = Q.w[i] * Q.w[j];
                for (int k = 0; k < Q.q; ++k) {
                    double xd[2], yd[2];
                    double jac = ss_dirs(ns, r, Q.t[i], Q.t[j], Q.t[k], xd, yd);
                    double D0 = xd[0] * X.e1[0] + xd[1] * X.e2[0] - yd[0] * Y.e1[0] - yd[1] * Y.e2[0];
                    double D1 = xd[0] * X.e1[1] + xd[1] * X.e2[1] - yd[0] * Y.e1[1] - yd[1] * Y.e2[1];
                    double D2 = xd[0] * X.e1[2] + xd[1] * X.e2[2] - yd[0] * Y.e1[2] - yd[1] * Y.e2[2];
                    double ir = rsqrt(D0 * D0 + D1 * D1 + D2 * D2);
                    double kern = (D0 * ny[0] + D1 * ny[1] + D2 * ny[2]) * ir * ir * ir;
                    const double f = wij * Q.w[k] * jac * kern;
                    out[0] += f * (0.5 - yd[0] * (1.0 / 3.0));
                    out[1] += f * ((yd[0] - yd[1]) * (1.0 / 3.0));
                    out[2] += f * (yd[1] * (1.0 / 3.0));
                }
            }
}

__device__ void pair_regular_dlp3(const Tri &X, const Tri &Y, const double ny[3], const QuadDev &Q, double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    for (int i = 0; i < Q.q; ++i) {
        const double u = Q.t[i];
        for (int j = 0; j < Q.q; ++j) {
            const double v = u * Q.t[j];
            const double wx = Q.w[i] * Q.w[j] * u;
            const double x0 = X.p[0] + u * X.e1[0] + v * X.e2[0];
            const double x1 = X.p[1] + u * X.e1[1] + v * X.e2[1];
            const double x2 = X.p[2] + u * X.e1[2] + v * X.e2[2];
            double in0 = 0.0, in1 = 0.0, in2 = 0.0;
            for (int k = 0; k < Q.q; ++k) {
                const double s = Q.t[k];
                const double ws = Q.w[k] * s;
                for (int l = 0; l < Q.q; ++l) {
                    const double sv = s * Q.t[l];
                    const double d0 = x0 - (Y.p[0] + s * Y.e1[0] + sv * Y.e2[0]);
                    const double d1 = x1 - (Y.p[1] + s * Y.e1[1] + sv * Y.e2[1]);
                    const double d2 = x2 - (Y.p[2] + s * Y.e1[2] + sv * Y.e2[2]);
                    const double ir = rsqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    const double f = (d0 * ny[0] + d1 * ny[1] + d2 * ny[2]) * ir * ir * ir;
                    const double wsl = ws * Q.w[l];
                    in0 += wsl * (f * (1.0 - s));
                    in1 += wsl * (f * (s - sv));
                    in2 += wsl * (f * sv);
                }
            }
            out[0] += wx * in0;
            out[1] += wx * in1;
            out[2] += wx * in2;
        }
    }
}

// K_{i, vertex} contributions of triangle tj for its three stored corners:
// val[slot] for the vertex in slot 0, 1, 2 of tj.
__device__ void dlp_triple(const GeoDev &g, int i, int tj, const QuadDev &Q, double val[3])
{
    int vi[3] = {g.t0[i], g.t1[i], g.t2[i]};
    int vj[3] = {g.t0[tj], g.t1[tj], g.t2[tj]};
    int oi[3], oj[3];
    int ns = pair_slots(vi, vj, oi, oj);
    Tri X, Y;
    load_tri(g, vi[oi[0]], vi[oi[1]], vi[oi[2]], X);
    load_tri(g, vj[oj[0]], vj[oj[1]], vj[oj[2]], Y);
    double ny[3] = {g.nx[tj], g.ny[tj], g.nz[tj]};
    double jj = tri_jac(X) * tri_jac(Y) * INV_4PI;
    double c3[3];
    if (ns == 0)
        pair_regular_dlp3(X, Y, ny, Q, c3);
    else
        dlp_touching3(ns, X, Y, ny, Q, c3);
    // quadrature corner c holds stored slot oj[c]
    for (int c = 0; c < 3; ++c) val[oj[c]] = c3[c] * jj;
}

// Column position of panel column c: walk the group's segments.
__device__ inline int panel_column(const RowPanelDev &d, int g, int c)
{
    int s = d.seg_ptr[g];
    const int s1 = d.seg_ptr[g + 1];
    while (s + 1 < s1 && c >= d.seg_len[s]) {
        c -= d.seg_len[s];
        ++s;
    }
    return d.seg_in[s] + c;
}

template <int KER>
__global__ __launch_bounds__(NT) void k_near_assemble(RowPanelDev d, const int32_t *__restrict__ rperm,
                                                      const int32_t *__restrict__ cperm, GeoDev geo,
                                                      QuadDev Q, double *__restrict__ vals)
{
    const int g = blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int ob = d.out_begin[g];
    const int64_t off = d.val_off[g];
    const int64_t n = (int64_t)nr * nc;
    for (int64_t e = threadIdx.x; e < n; e += NT) {
        const int r = (int)(e / nc), c = (int)(e % nc);
        const int i = rperm[ob + r];
        const int j = cperm[panel_column(d, g, c)];
        double v;
        if (KER == 0) {
            v = slp_entry(geo, i, j, Q);
        } else {
            v = 0.0;
            for (int64_t a = geo.vt_ptr[j]; a < geo.vt_ptr[j + 1]; ++a) {
                const int tj = geo.vt_idx[a];
                const int slot = (geo.t0[tj] == j) ? 0 : (geo.t1[tj] == j) ? 1 : 2;
                v += dlp_part(geo, i, tj, slot, Q);
            }
        }
        vals[off + e] = v;
    }
}

// Double-layer nearfield with every triangle pair integrated once: for each
// row i of the group, the pair integrals (i, tau) for all triangles tau around
// the group's column vertices (the sorted list lst[lptr[g] ..]) are computed
// with all three corner weights into LDS, CH triangles at a time; then every
// entry (i, j) sums the contributions of the triangles around vertex j in the
// vertex's own order.
constexpr int DLP_CH = 1536;

__global__ __launch_bounds__(NT) void k_near_assemble_dlp(RowPanelDev d, const int32_t *__restrict__ rperm,
                                                          const int32_t *__restrict__ cperm, GeoDev geo, QuadDev Q,
                                                          const int64_t *__restrict__ lptr,
                                                          const int32_t *__restrict__ lst, double *__restrict__ vals)
{
    __shared__ int32_t tri[DLP_CH];
    __shared__ double w[3 * DLP_CH];
    const int g = blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int ob = d.out_begin[g];
    const int64_t off = d.val_off[g];
    const int64_t l0 = lptr[g];
    const int nl = (int)(lptr[g + 1] - l0);
    for (int r = 0; r < nr; ++r) {
        const int i = rperm[ob + r];
        for (int h0 = 0; h0 < nl; h0 += DLP_CH) {
            const int hl = min(DLP_CH, nl - h0);
            __syncthreads();  // the previous chunk has been read
            for (int e = threadIdx.x; e < hl; e += NT) {
                const int tj = lst[l0 + h0 + e];
                tri[e] = tj;
                dlp_triple(geo, i, tj, Q, w + 3 * e);
            }
            __syncthreads();
            for (int c = threadIdx.x; c < nc; c += NT) {
                const int j = cperm[panel_column(d, g, c)];
                double v = 0.0;
                for (int64_t a = geo.vt_ptr[j]; a < geo.vt_ptr[j + 1]; ++a) {
                    const int tj = geo.vt_idx[a];
                    int lo = 0, hi = hl;  // first position with tri[pos] >= tj
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (tri[mid] < tj)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    if (lo < hl && tri[lo] == tj) {
                        const int slot = (geo.t0[tj] == j) ? 0 : (geo.t1[tj] == j) ? 1 : 2;
                        v += w[3 * lo + slot];
                    }
                }
                double *dst = vals + off + (int64_t)r * nc + c;
                *dst = h0 == 0 ? v : *dst + v;
            }
        }
    }
}

// ===================================================================
//  Interpolation: Lagrange polynomials on Chebyshev points (Section 3)
// ===================================================================

// ell_a(z) on the m points pts.
__device__ inline double lag1(const double *pts, int m, int a, double z)
{
    double v = 1.0;
    for (int b = 0; b < m; ++b)
        if (b != a) v *= (z - pts[b]) / (pts[a] - pts[b]);
    return v;
}

// d ell_a / dz.
__device__ inline double lag1d(const double *pts, int m, int a, double z)
{
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
        if (k == a) continue;
        double v = 1.0 / (pts[a] - pts[k]);
        for (int b = 0; b < m; ++b)
            if (b != a && b != k) v *= (z - pts[b]) / (pts[a] - pts[b]);
        s += v;
    }
    return s;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_leaf_basis(bool dlp_cols, RowPanelDev d,
                                                   const int32_t *__restrict__ perm,
                                                   const double *__restrict__ axes, int m,
                                                   GeoDev geo, QuadDev Q, T *__restrict__ vals)
{
    const int g = blockIdx.x;
    const int cl = d.tag[g];
    const int k = d.nrows[g], nc = d.ncols[g];
    const int in0 = d.seg_in[d.seg_ptr[g]];
    const int64_t off = d.val_off[g];
    __shared__ double ax[3 * MMAX];
    if (threadIdx.x < 3 * m) ax[threadIdx.x] = axes[(int64_t)cl * 3 * m + threadIdx.x];
    __syncthreads();
    const int64_t n = (int64_t)k * nc;
    for (int64_t e = threadIdx.x; e < n; e += NT) {
        const int nu = (int)(e / nc), r = (int)(e % nc);
        const int n1 = nu % m, n2 = (nu / m) % m, n3 = nu / (m * m);
        const int idx = perm[in0 + r];
        double acc = 0.0;
        auto one_triangle = [&](int tri, int slot) {
            Tri tr;
            load_tri(geo, geo.t0[tri], geo.t1[tri], geo.t2[tri], tr);
            const double J = tri_jac(tr);
            double s = 0.0;
            for (int a = 0; a < Q.q; ++a) {
                const double u = Q.t[a];
                for (int b = 0; b < Q.q; ++b) {
                    const double v = u * Q.t[b];
                    const double w = Q.w[a] * Q.w[b] * u;
                    const double x = tr.p[0] + u * tr.e1[0] + v * tr.e2[0];
                    const double y = tr.p[1] + u * tr.e1[1] + v * tr.e2[1];
                    const double z = tr.p[2] + u * tr.e1[2] + v * tr.e2[2];
                    const double l1 = lag1(ax, m, n1, x), l2 = lag1(ax + m, m, n2, y),
                                 l3 = lag1(ax + 2 * m, m, n3, z);
                    if (slot < 0) {
                        s += w * l1 * l2 * l3;
                    } else {
                        const double lam = (slot == 0) ? 1.0 - u : (slot == 1) ? u - v : v;
                        const double g1 = lag1d(ax, m, n1, x) * l2 * l3;
                        const double g2 = l1 * lag1d(ax + m, m, n2, y) * l3;
                        const double g3 = l1 * l2 * lag1d(ax + 2 * m, m, n3, z);
                        s += w * lam * (g1 * geo.nx[tri] + g2 * geo.ny[tri] + g3 * geo.nz[tri]);
                    }
                }
            }
            acc += J * s;
        };
        if (!dlp_cols) {
            one_triangle(idx, -1);
        } else {
            for (int64_t a = geo.vt_ptr[idx]; a < geo.vt_ptr[idx + 1]; ++a) {
                const int tri = geo.vt_idx[a];
                const int slot = (geo.t0[tri] == idx) ? 0 : (geo.t1[tri] == idx) ? 1 : 2;
                one_triangle(tri, slot);
            }
        }
        vals[off + nu * (int64_t)nc + r] = (T)acc;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_transfer(RowPanelDev d, const double *__restrict__ axes,
                                                 int m, T *__restrict__ vals)
{
    const int g = blockIdx.x;
    const int t = d.tag[g];
    const int k = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int s0 = d.seg_ptr[g], s1 = d.seg_ptr[g + 1];
    const double *pt = axes + (int64_t)t * 3 * m;
    const int64_t n = (int64_t)k * nc;
    for (int64_t e = threadIdx.x; e < n; e += NT) {
        const int nu = (int)(e / nc);
        int c = (int)(e % nc);
        int s = s0;
        while (s + 1 < s1 && c >= d.seg_len[s]) {
            c -= d.seg_len[s];
            ++s;
        }
        const double *pc = axes + (int64_t)d.seg_tag[s] * 3 * m;
        const int mu = c;
        const double v = lag1(pt, m, nu % m, pc[mu % m]) *
                         lag1(pt + m, m, (nu / m) % m, pc[m + (mu / m) % m]) *
                         lag1(pt + 2 * m, m, nu / (m * m), pc[2 * m + mu / (m * m)]);
        vals[off + e] = (T)v;
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_coupling(RowPanelDev d, const double *__restrict__ raxes,
                                                 const double *__restrict__ caxes, int m,
                                                 T *__restrict__ vals)
{
    const int g = blockIdx.x;
    const int t = d.tag[g];
    const int k = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int s0 = d.seg_ptr[g], s1 = d.seg_ptr[g + 1];
    const double *pt = raxes + (int64_t)t * 3 * m;
    const int64_t n = (int64_t)k * nc;
    for (int64_t e = threadIdx.x; e < n; e += NT) {
        const int nu = (int)(e / nc);
        int c = (int)(e % nc);
        int s = s0;
        while (s + 1 < s1 && c >= d.seg_len[s]) {
            c -= d.seg_len[s];
            ++s;
        }
        const double *ps = caxes + (int64_t)d.seg_tag[s] * 3 * m;
        const int mu = c;
        const double dx = pt[nu % m] - ps[mu % m];
        const double dy = pt[m + (nu / m) % m] - ps[m + (mu / m) % m];
        const double dz = pt[2 * m + nu / (m * m)] - ps[2 * m + mu / (m * m)];
        vals[off + e] = (T)(INV_4PI * rsqrt(dx * dx + dy * dy + dz * dz));
    }
}

// ===================================================================
//  Shape derivatives (frozen trees, boxes and interpolation points)
// ===================================================================

// d|e1 x e2| / d(corner c) for the parametrisation P0 + u1 e1 + u2 e2,
// e1 = P1 - P0, e2 = P2 - P1: with n the unit normal, dJ = (e2 x n).de1 +
// (n x e1).de2.
__device__ inline void jac_grad(const Tri &T, double J, double out[3][3])
{
    double n[3] = {T.e1[1] * T.e2[2] - T.e1[2] * T.e2[1], T.e1[2] * T.e2[0] - T.e1[0] * T.e2[2],
                   T.e1[0] * T.e2[1] - T.e1[1] * T.e2[0]};
    for (int d = 0; d < 3; ++d) n[d] /= J;
    const double a[3] = {T.e2[1] * n[2] - T.e2[2] * n[1], T.e2[2] * n[0] - T.e2[0] * n[2],
                         T.e2[0] * n[1] - T.e2[1] * n[0]};  // e2 x n
    const double b[3] = {n[1] * T.e1[2] - n[2] * T.e1[1], n[2] * T.e1[0] - n[0] * T.e1[2],
                         n[0] * T.e1[1] - n[1] * T.e1[0]};  // n x e1
    for (int d = 0; d < 3; ++d) {
        out[0][d] = -a[d];
        out[1][d] = a[d] - b[d];
        out[2][d] = b[d];
    }
}

// Adds w * dG_ij / d(vertex coordinates) into g (3 arrays), G_ij being the
// regularised-quadrature value of slp_entry: derivative of the same rule with
// respect to the corners, through the Jacobians and through x - y (the xi
// integral of the touching rules again in closed form).
__device__ void slp_entry_grad(const GeoDev &g, int i, int j, const QuadDev &Q, double w, double *gx,
                               double *gy, double *gz)
{
    int vi[3] = {g.t0[i], g.t1[i], g.t2[i]};
    int vj[3] = {g.t0[j], g.t1[j], g.t2[j]};
    int oi[3], oj[3];
    const int ns = pair_slots(vi, vj, oi, oj);
    Tri X, Y;
    load_tri(g, vi[oi[0]], vi[oi[1]], vi[oi[2]], X);
    load_tri(g, vj[oj[0]], vj[oj[1]], vj[oj[2]], Y);
    double I = 0.0, dX[3][3] = {{0}}, dY[3][3] = {{0}};
    if (ns == 0) {
        for (int a = 0; a < Q.q; ++a) {
            const double u = Q.t[a];
            for (int b = 0; b < Q.q; ++b) {
                const double v = u * Q.t[b];
                const double wx = Q.w[a] * Q.w[b] * u;
                const double lx[3] = {1.0 - u, u - v, v};
                double x[3];
                for (int d = 0; d < 3; ++d) x[d] = X.p[d] + u * X.e1[d] + v * X.e2[d];
                for (int c = 0; c < Q.q; ++c) {
                    const double s = Q.t[c];
                    for (int e = 0; e < Q.q; ++e) {
                        const double sv = s * Q.t[e];
                        const double wq = wx * Q.w[c] * Q.w[e] * s;
                        const double ly[3] = {1.0 - s, s - sv, sv};
                        double dd[3];
                        for (int d = 0; d < 3; ++d) dd[d] = x[d] - (Y.p[d] + s * Y.e1[d] + sv * Y.e2[d]);
                        const double ir = rsqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
                        const double ir3 = wq * ir * ir * ir;
                        I += wq * ir;
                        for (int k = 0; k < 3; ++k)
                            for (int d = 0; d < 3; ++d) {
                                dX[k][d] -= lx[k] * dd[d] * ir3;
                                dY[k][d] += ly[k] * dd[d] * ir3;
                            }
                    }
                }
            }
        }
    } else {
        const int nreg = (ns == 3) ? 6 : (ns == 2) ? 5 : 2;
        for (int r = 0; r < nreg; ++r)
            for (int a = 0; a < Q.q; ++a)
                for (int b = 0; b < Q.q; ++b)
                    for (int c = 0; c < Q.q; ++c) {
                        double xd[2], yd[2];
                        const double jac = ss_dirs(ns, r, Q.t[a], Q.t[b], Q.t[c], xd, yd);
                        const double wq = Q.w[a] * Q.w[b] * Q.w[c] * jac;
                        double D[3];
                        for (int d = 0; d < 3; ++d)
                            D[d] = xd[0] * X.e1[d] + xd[1] * X.e2[d] - yd[0] * Y.e1[d] - yd[1] * Y.e2[d];
                        const double ir = rsqrt(D[0] * D[0] + D[1] * D[1] + D[2] * D[2]);
                        const double ir3 = wq * ir * ir * ir;
                        I += wq * ir * (1.0 / 3.0);
                        // int_0^1 xi * barycentric(xi X) d xi
                        const double lx[3] = {0.5 - xd[0] * (1.0 / 3.0), (xd[0] - xd[1]) * (1.0 / 3.0),
                                              xd[1] * (1.0 / 3.0)};
                        const double ly[3] = {0.5 - yd[0] * (1.0 / 3.0), (yd[0] - yd[1]) * (1.0 / 3.0),
                                              yd[1] * (1.0 / 3.0)};
                        for (int k = 0; k < 3; ++k)
                            for (int d = 0; d < 3; ++d) {
                                dX[k][d] -= lx[k] * D[d] * ir3;
                                dY[k][d] += ly[k] * D[d] * ir3;
                            }
                    }
    }
    const double Jx = tri_jac(X), Jy = tri_jac(Y);
    double gJx[3][3], gJy[3][3];
    jac_grad(X, Jx, gJx);
    jac_grad(Y, Jy, gJy);
    const double s = w * INV_4PI;
    for (int k = 0; k < 3; ++k) {
        const int vx = vi[oi[k]], vy = vj[oj[k]];
        double ax[3], ay[3];
        for (int d = 0; d < 3; ++d) {
            ax[d] = s * (gJx[k][d] * Jy * I + Jx * Jy * dX[k][d]);
            ay[d] = s * (Jx * gJy[k][d] * I + Jx * Jy * dY[k][d]);
        }
        atomicAdd(gx + vx, ax[0]);
        atomicAdd(gy + vx, ax[1]);
        atomicAdd(gz + vx, ax[2]);
        atomicAdd(gx + vy, ay[0]);
        atomicAdd(gy + vy, ay[1]);
        atomicAdd(gz + vy, ay[2]);
    }
}

// Near-field part of d(x^T G y)/dV: every stored entry (i, j) contributes
// x_i y_j dG_ij.  xp, yp in cluster order.
__global__ __launch_bounds__(NT) void k_near_grad(RowPanelDev d, const int32_t *__restrict__ perm, GeoDev geo,
                                                  QuadDev Q, const double *__restrict__ xp,
                                                  const double *__restrict__ yp, double *gx, double *gy,
                                                  double *gz)
{
    const int g = blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int ob = d.out_begin[g];
    const int64_t n = (int64_t)nr * nc;
    for (int64_t e = threadIdx.x; e < n; e += NT) {
        const int r = (int)(e / nc), c = (int)(e % nc);
        const int cpos = panel_column(d, g, c);
        const double w = xp[ob + r] * yp[cpos];
        if (w == 0.0) continue;
        slp_entry_grad(geo, perm[ob + r], perm[cpos], Q, w, gx, gy, gz);
    }
}

// Far-field part through the leaf bases: for triangle i of leaf t with
// coefficients c = x_i a_t(y) + y_i a_t(x) (a = leaf coefficients of the
// partial products), adds d/dV of int_{tau_i} sum_nu c_nu L_{t,nu}.
template <typename F>
__global__ __launch_bounds__(NT) void k_leaf_grad(RowPanelDev d, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ axes, int m, GeoDev geo, QuadDev Q,
                                                  const F *__restrict__ ax, const F *__restrict__ ay,
                                                  const double *__restrict__ xp, const double *__restrict__ yp,
                                                  double *gx, double *gy, double *gz)
{
    const int g = blockIdx.x;
    const int cl = d.tag[g];
    const int k = d.nrows[g], n = d.ncols[g];
    const int in0 = d.seg_in[d.seg_ptr[g]];
    const int hb = d.out_begin[g];
    __shared__ double axs[3 * MMAX];
    if (threadIdx.x < 3 * m) axs[threadIdx.x] = axes[(int64_t)cl * 3 * m + threadIdx.x];
    __syncthreads();
    for (int r = threadIdx.x; r < n; r += NT) {
        const int tri = perm[in0 + r];
        const double xr = xp[in0 + r], yr = yp[in0 + r];
        Tri T;
        load_tri(geo, geo.t0[tri], geo.t1[tri], geo.t2[tri], T);
        const double J = tri_jac(T);
        double S = 0.0, Tc[3][3] = {{0}};
        for (int a = 0; a < Q.q; ++a) {
            const double u = Q.t[a];
            for (int b = 0; b < Q.q; ++b) {
                const double v = u * Q.t[b];
                const double wq = Q.w[a] * Q.w[b] * u;
                double p[3];
                for (int dd = 0; dd < 3; ++dd) p[dd] = T.p[dd] + u * T.e1[dd] + v * T.e2[dd];
                double l[3][MMAX], dl[3][MMAX];
                for (int dd = 0; dd < 3; ++dd)
                    for (int q = 0; q < m; ++q) {
                        l[dd][q] = lag1(axs + dd * m, m, q, p[dd]);
                        dl[dd][q] = lag1d(axs + dd * m, m, q, p[dd]);
                    }
                double f = 0.0, gf[3] = {0.0, 0.0, 0.0};
                for (int nu = 0; nu < k; ++nu) {
                    const double cnu = xr * (double)ay[hb + nu] + yr * (double)ax[hb + nu];
                    const int n1 = nu % m, n2 = (nu / m) % m, n3 = nu / (m * m);
                    f += cnu * l[0][n1] * l[1][n2] * l[2][n3];
                    gf[0] += cnu * dl[0][n1] * l[1][n2] * l[2][n3];
                    gf[1] += cnu * l[0][n1] * dl[1][n2] * l[2][n3];
                    gf[2] += cnu * l[0][n1] * l[1][n2] * dl[2][n3];
                }
                S += wq * f;
                const double lam[3] = {1.0 - u, u - v, v};
                for (int c = 0; c < 3; ++c)
                    for (int dd = 0; dd < 3; ++dd) Tc[c][dd] += wq * lam[c] * gf[dd];
            }
        }
        double gJ[3][3];
        jac_grad(T, J, gJ);
        const int vv[3] = {geo.t0[tri], geo.t1[tri], geo.t2[tri]};
        for (int c = 0; c < 3; ++c) {
            atomicAdd(gx + vv[c], gJ[c][0] * S + J * Tc[c][0]);
            atomicAdd(gy + vv[c], gJ[c][1] * S + J * Tc[c][1]);
            atomicAdd(gz + vv[c], gJ[c][2] * S + J * Tc[c][2]);
        }
    }
}

// ===================================================================
//  Panel products
// ===================================================================

template <typename T> struct Acc { using type = double; };
template <> struct Acc<float> { using type = float; };
template <> struct Acc<bf16_t> { using type = float; };

template <typename A> __device__ inline A wave_sum(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

constexpr int CHUNK = 4096;  // largest number of input columns staged in LDS per pass

template <typename T> __device__ inline T stream_load(const T *p) { return __builtin_nontemporal_load(p); }

// Segment descriptors of a group held in LDS by the row-panel kernel (groups
// with more segments read them from global memory).
template <int NW> constexpr int max_lds_segments() { return NW == 1 ? 128 : 512; }

// Index of the segment holding panel column col: the last s in [0, n) with
// c0[s] <= col (a zero-length segment shares its start with the next one).
__device__ inline int find_segment(const int32_t *c0, int n, int col)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (c0[mid] <= col)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// One workgroup of NW waves per group.  The group's segment descriptors go to
// LDS; each column chunk of the input is gathered into LDS with every thread
// issuing up to 8 independent loads (segment found by binary search), then
// every wave takes RW rows at a time and streams them with coalesced
// non-temporal loads (4 column blocks of 64 per row, 4*RW loads in flight per
// lane; the last < 4 blocks of a row are issued together under per-lane
// predicates); rows past the end repeat the last row, whose sums are dropped
// (cheaper than branching around them).
// Per-row partial sums live in LDS across chunks.
template <typename VT, typename XT, typename YT, int ROLE, int NW, int RW>
__global__ __launch_bounds__(NW * 64) void k_rowpanel(RowPanelDev d, int g0, int chunk,
                                                      const VT *__restrict__ vals,
                                                      const XT *__restrict__ x, YT *__restrict__ y,
                                                      int accumulate)
{
    using A = typename Acc<VT>::type;
    constexpr int NTH = NW * 64;
    constexpr int MAXSEG = max_lds_segments<NW>();
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    A *racc = xs + chunk;
    __shared__ int32_t lds_c0[MAXSEG], lds_in[MAXSEG];
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sb = d.seg_ptr[g], nseg = d.seg_ptr[g + 1] - sb;
    const int32_t *c0s = d.seg_c0 + sb, *ins = d.seg_in + sb;
    if (nseg <= MAXSEG) {
        for (int t = threadIdx.x; t < nseg; t += NTH) {
            lds_c0[t] = c0s[t];
            lds_in[t] = ins[t];
        }
        c0s = lds_c0;
        ins = lds_in;
    }
    __syncthreads();

    for (int c0 = 0; c0 < nc; c0 += chunk) {
        const int clen = min(chunk, nc - c0);
        for (int e0 = threadIdx.x; e0 < clen; e0 += 8 * NTH) {
            A v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * NTH;
                v[q] = 0;
                if (e < clen) {
                    const int col = c0 + e;
                    const int sg = find_segment(c0s, nseg, col);
                    v[q] = (A)x[ins[sg] + (col - c0s[sg])];
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (e0 + q * NTH < clen) xs[e0 + q * NTH] = v[q];
        }
        __syncthreads();
        for (int r = RW * wave; r < nr; r += RW * NW) {
            A acc[RW][4];
#pragma unroll
            for (int i = 0; i < RW; ++i)
#pragma unroll
                for (int k = 0; k < 4; ++k) acc[i][k] = 0;
            const VT *rows[RW];
#pragma unroll
            for (int i = 0; i < RW; ++i) rows[i] = vals + off + (int64_t)min(r + i, nr - 1) * nc + c0;
            int c = lane;
            for (; c + 192 < clen; c += 256) {
                A xv[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) xv[k] = xs[c + 64 * k];
#pragma unroll
                for (int i = 0; i < RW; ++i)
#pragma unroll
                    for (int k = 0; k < 4; ++k) acc[i][k] += (A)stream_load(rows[i] + c + 64 * k) * xv[k];
            }
            if (c < clen) {  // fewer than 4 column blocks left: issue them together
                A xv[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) xv[k] = (c + 64 * k < clen) ? xs[c + 64 * k] : A(0);
#pragma unroll
                for (int i = 0; i < RW; ++i) {
                    VT p[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) p[k] = (c + 64 * k < clen) ? stream_load(rows[i] + c + 64 * k) : VT(0);
#pragma unroll
                    for (int k = 0; k < 3; ++k) acc[i][k] += (A)p[k] * xv[k];
                }
            }
#pragma unroll
            for (int i = 0; i < RW; ++i) {
                const A sum = wave_sum((acc[i][0] + acc[i][1]) + (acc[i][2] + acc[i][3]));
                if (lane == 0 && r + i < nr) racc[r + i] = (c0 == 0) ? sum : racc[r + i] + sum;
            }
        }
        __syncthreads();
    }
    const int ob = d.out_begin[g];
    for (int r = threadIdx.x; r < nr; r += NTH) {
        const A v = (nc > 0) ? racc[r] : A(0);
        if (accumulate)
            y[ob + r] = (YT)((A)y[ob + r] + v);
        else
            y[ob + r] = (YT)v;
    }
}

// One workgroup per output segment: lanes over output entries (64 at a time),
// waves over the rows of all contributing blocks, partial sums reduced in LDS.
template <typename VT, typename XT, typename YT, int ROLE>
__global__ __launch_bounds__(NT) void k_colpanel(ColPanelDev d, int g0, const VT *__restrict__ vals,
                                                 const XT *__restrict__ x, YT *__restrict__ y)
{
    using A = typename Acc<VT>::type;
    constexpr int NW = NT / 64;
    __shared__ A red[NW][64];
    const int g = g0 + blockIdx.x;
    const int ob = d.out_begin[g], ol = d.out_len[g];
    const int b0 = d.blk_ptr[g], b1 = d.blk_ptr[g + 1];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int jc = 0; jc < ol; jc += 64) {
        const int j = jc + lane;
        const bool valid = j < ol;
        A acc = 0;
        int base = 0;
        for (int b = b0; b < b1; ++b) {
            const int nrb = d.b_nrows[b];
            const int64_t stride = d.b_stride[b];
            const VT *col = vals + d.b_val_off[b] + d.b_c0[b] + j;
            const XT *xin = x + d.b_in[b];
            int i = (wave - base) % NW;
            if (i < 0) i += NW;
            if (valid) {
                A a1 = 0, a2 = 0, a3 = 0;
                for (; i + 3 * NW < nrb; i += 4 * NW) {
                    const VT v0 = stream_load(col + i * stride);
                    const VT v1 = stream_load(col + (i + NW) * stride);
                    const VT v2 = stream_load(col + (i + 2 * NW) * stride);
                    const VT v3 = stream_load(col + (i + 3 * NW) * stride);
                    acc += (A)v0 * (A)xin[i];
                    a1 += (A)v1 * (A)xin[i + NW];
                    a2 += (A)v2 * (A)xin[i + 2 * NW];
                    a3 += (A)v3 * (A)xin[i + 3 * NW];
                }
                for (; i < nrb; i += NW) acc += (A)stream_load(col + i * stride) * (A)xin[i];
                acc += (a1 + a2) + a3;
            }
            base += nrb;
        }
        red[wave][lane] = acc;
        __syncthreads();
        if (wave == 0 && valid) {
            A s = red[0][lane];
#pragma unroll
            for (int w = 1; w < NW; ++w) s += red[w][lane];
            y[ob + j] = (YT)((A)y[ob + j] + s);
        }
        __syncthreads();
    }
}

__global__ void k_gather(const int32_t *__restrict__ perm, int64_t n, int nrhs,
                         const double *__restrict__ x, int64_t ldx, double *__restrict__ xp)
{
    const int64_t tot = n * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, k = e % n;
        xp[e] = x[perm[k] + c * ldx];
    }
}

__global__ void k_scatter_add(const int32_t *__restrict__ perm, int64_t n, int nrhs, double alpha,
                              const double *__restrict__ yp, const double *__restrict__ yp2,
                              double *__restrict__ y, int64_t ldy)
{
    const int64_t tot = n * nrhs;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t c = e / n, k = e % n;
        const double v = yp2 ? yp[e] + yp2[e] : yp[e];
        y[perm[k] + c * ldy] += alpha * v;
    }
}

template <typename T> __global__ void k_fill_zero(T *__restrict__ p, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = T(0);
}

}  // namespace

// ===================================================================
//  Launchers
// ===================================================================

void launch_near_assemble(h2b_kernel kernel, const RowPanels &rp, const int32_t *rperm,
                          const int32_t *cperm, const GeoDev &geo, const QuadDev &quad,
                          double *vals, hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    if (kernel == H2B_SLP)
        hipLaunchKernelGGL(k_near_assemble<0>, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, rperm,
                           cperm, geo, quad, vals);
    else
        hipLaunchKernelGGL(k_near_assemble<1>, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, rperm,
                           cperm, geo, quad, vals);
    hip_check(hipGetLastError(), "nearfield assembly launch");
}

void launch_near_assemble_dlp(const RowPanels &rp, const int64_t *lptr, const int32_t *lst, const int32_t *rperm,
                              const int32_t *cperm, const GeoDev &geo, const QuadDev &quad, double *vals,
                              hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_near_assemble_dlp, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, rperm, cperm, geo, quad,
                       lptr, lst, vals);
    hip_check(hipGetLastError(), "double-layer nearfield assembly launch");
}

void launch_near_grad(const RowPanels &rp, const int32_t *perm, const GeoDev &geo, const QuadDev &quad,
                      const double *xp, const double *yp, double *gx, double *gy, double *gz, hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_near_grad, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, perm, geo, quad, xp, yp, gx, gy,
                       gz);
    hip_check(hipGetLastError(), "nearfield gradient launch");
}

template <typename F>
void launch_leaf_grad(const RowPanels &leaf, const int32_t *perm, const double *axes, int m, const GeoDev &geo,
                      const QuadDev &quad, const F *ax, const F *ay, const double *xp, const double *yp,
                      double *gx, double *gy, double *gz, hipStream_t st)
{
    if (leaf.ngroups() == 0) return;
    hipLaunchKernelGGL(k_leaf_grad<F>, dim3(leaf.ngroups()), dim3(NT), 0, st, leaf.dev, perm, axes, m, geo, quad,
                       ax, ay, xp, yp, gx, gy, gz);
    hip_check(hipGetLastError(), "leaf gradient launch");
}

template <typename T>
void launch_leaf_basis(bool dlp_cols, const RowPanels &rp, const int32_t *perm, const double *axes,
                       int m, const GeoDev &geo, const QuadDev &quad, T *vals, hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_leaf_basis<T>, dim3(rp.ngroups()), dim3(NT), 0, st, dlp_cols, rp.dev, perm,
                       axes, m, geo, quad, vals);
    hip_check(hipGetLastError(), "leaf basis launch");
}

template <typename T>
void launch_transfer(const RowPanels &rp, const double *axes, int m, T *vals, hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_transfer<T>, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, axes, m, vals);
    hip_check(hipGetLastError(), "transfer launch");
}

template <typename T>
void launch_coupling(const RowPanels &rp, const double *raxes, const double *caxes, int m, T *vals,
                     hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_coupling<T>, dim3(rp.ngroups()), dim3(NT), 0, st, rp.dev, raxes, caxes, m, vals);
    hip_check(hipGetLastError(), "coupling launch");
}

// Narrow panels (leaf and transfer matrices, at most 128 input columns): one
// wave per group, input in LDS, eight rows per iteration so that eight
// independent loads per lane are in flight before the reductions.
template <typename VT, typename XT, typename YT, int ROLE>
__global__ __launch_bounds__(64) void k_rowpanel_narrow(RowPanelDev d, int g0, const VT *__restrict__ vals,
                                                        const XT *__restrict__ x, YT *__restrict__ y,
                                                        int accumulate)
{
    using A = typename Acc<VT>::type;
    __shared__ A xs[128];
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int lane = threadIdx.x;
    {
        int filled = 0;
        for (int s = d.seg_ptr[g]; s < d.seg_ptr[g + 1]; ++s) {
            const int len = d.seg_len[s];
            const XT *src = x + d.seg_in[s];
            for (int j = lane; j < len; j += 64) xs[filled + j] = (A)src[j];
            filled += len;
        }
    }
    __syncthreads();
    const A x0 = (lane < nc) ? xs[lane] : A(0);
    const A x1 = (lane + 64 < nc) ? xs[lane + 64] : A(0);
    const int ob = d.out_begin[g];
    for (int r = 0; r < nr; r += 8) {
        A acc[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            acc[q] = 0;
            const int rr = min(r + q, nr - 1);
            const VT *row = vals + off + (int64_t)rr * nc;
            if (lane < nc) acc[q] += (A)row[lane] * x0;
            if (lane + 64 < nc) acc[q] += (A)row[lane + 64] * x1;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const A v = wave_sum(acc[q]);
            if (lane == 0 && r + q < nr) {
                if (accumulate)
                    y[ob + r + q] = (YT)((A)y[ob + r + q] + v);
                else
                    y[ob + r + q] = (YT)v;
            }
        }
    }
}

template <typename VT, typename XT, typename YT, int ROLE, int NW, int RW>
static void rowpanel_nw(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y, int acc,
                        hipStream_t st)
{
    using A = typename Acc<VT>::type;
    int chunk = std::min(CHUNK, std::max(64, (rp.max_ncols + 63) / 64 * 64));
    if (NW == 1) chunk = std::min(chunk, 1024);
    const size_t shm = sizeof(A) * ((size_t)chunk + (size_t)std::max(rp.max_nrows, 1));
    hipLaunchKernelGGL((k_rowpanel<VT, XT, YT, ROLE, NW, RW>), dim3(g1 - g0), dim3(NW * 64), shm, st, rp.dev,
                       g0, chunk, vals, x, y, acc);
}

template <typename VT, typename XT, typename YT, int ROLE>
static void rowpanel_role(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y, int acc,
                          hipStream_t st)
{
    // small panels (recompressed coupling, leaf and transfer matrices) get one
    // wave per group taking four rows at a time, so that many groups stream
    // concurrently; tall panels (near field) share the staged input among four
    // waves taking two rows each
    const double rows_per_group = (double)rp.total / std::max<int64_t>(1, (int64_t)rp.ngroups()) /
                                  std::max(1.0, (double)rp.max_ncols);
    if (rp.max_ncols <= 128 && (ROLE == 0 || ROLE == 1)) {
        hipLaunchKernelGGL((k_rowpanel_narrow<VT, XT, YT, ROLE>), dim3(g1 - g0), dim3(64), 0, st, rp.dev, g0, vals,
                           x, y, acc);
        return;
    }
    if (rp.max_nrows <= 32 || rows_per_group < 16)
        rowpanel_nw<VT, XT, YT, ROLE, 1, 4>(rp, g0, g1, vals, x, y, acc, st);
    else
        rowpanel_nw<VT, XT, YT, ROLE, 4, 2>(rp, g0, g1, vals, x, y, acc, st);
}

template <typename VT, typename XT, typename YT>
void launch_rowpanel(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y,
                     bool accumulate, hipStream_t st, Role role)
{
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
    switch (role) {
    case Role::Leaf: rowpanel_role<VT, XT, YT, 0>(rp, g0, g1, vals, x, y, acc, st); break;
    case Role::Transfer: rowpanel_role<VT, XT, YT, 1>(rp, g0, g1, vals, x, y, acc, st); break;
    case Role::Coupling: rowpanel_role<VT, XT, YT, 2>(rp, g0, g1, vals, x, y, acc, st); break;
    default: rowpanel_role<VT, XT, YT, 3>(rp, g0, g1, vals, x, y, acc, st); break;
    }
    hip_check(hipGetLastError(), "row panel launch");
}

// Transposed product of narrow panels (leaf and transfer matrices): one wave per
// output segment.  An output of ol <= 32 entries is covered S = 2 or 4 times
// (lanes j + L*slice, L = 64/S lanes per slice), each slice taking every S-th
// row of the blocks, so that more loads are in flight and each lane's chain is
// S times shorter; the slices are summed with cross-lane shuffles.
template <typename VT, typename XT, typename YT, int ROLE>
__global__ __launch_bounds__(64) void k_colpanel_narrow(ColPanelDev d, int g0, const VT *__restrict__ vals,
                                                        const XT *__restrict__ x, YT *__restrict__ y,
                                                        int accumulate)
{
    using A = typename Acc<VT>::type;
    const int g = g0 + blockIdx.x;
    const int ob = d.out_begin[g], ol = d.out_len[g];
    const int b0 = d.blk_ptr[g], b1 = d.blk_ptr[g + 1];
    const int L = ol <= 16 ? 16 : ol <= 32 ? 32 : 64;
    const int S = 64 / L;
    const int lane = threadIdx.x, slice = lane / L;
    for (int j0 = 0; j0 < ol; j0 += L) {
        const int j = j0 + (lane % L);
        const bool valid = j < ol;
        A acc = 0;
        if (valid) {
            for (int b = b0; b < b1; ++b) {
                const VT *col = vals + d.b_val_off[b] + d.b_c0[b] + j;
                const int64_t stride = d.b_stride[b];
                const XT *v = x + d.b_in[b];
                const int n = d.b_nrows[b];
                A a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                int i = slice;
                for (; i + 7 * S < n; i += 8 * S) {
#pragma unroll
                    for (int q = 0; q < 8; ++q) a[q] += (A)col[(i + q * S) * stride] * (A)v[i + q * S];
                }
                for (; i < n; i += S) a[0] += (A)col[i * stride] * (A)v[i];
                acc += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
            }
        }
        for (int o = L; o < 64; o <<= 1) acc += __shfl_xor(acc, o, 64);
        if (valid && slice == 0) y[ob + j] = accumulate ? (YT)((A)y[ob + j] + acc) : (YT)acc;
    }
}

// Transposed product of whole narrow panels (backward transformation through
// leaf and transfer matrices): one wave per group, lanes over the panel's
// columns, the group's input x[out_begin ..] (one entry per row) in LDS, 16
// rows in flight; column c goes to the entry of its segment.  The outputs of
// different groups are disjoint (children of distinct parents, distinct
// leaves), so no reduction across groups is needed.  Invalid lanes (c >= nc)
// read column 0 and discard the sum.
template <typename VT, typename XT, typename YT, int ROLE>
__global__ __launch_bounds__(64) void k_rowpanelT_narrow(RowPanelDev d, int g0, const VT *__restrict__ vals,
                                                         const XT *__restrict__ x, YT *__restrict__ y)
{
    using A = typename Acc<VT>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    A *xs = reinterpret_cast<A *>(smem_raw);
    const int g = g0 + blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int lane = threadIdx.x;
    const XT *xin = x + d.out_begin[g];
    for (int i = lane; i < nr; i += 64) xs[i] = (A)xin[i];
    __syncthreads();
    const int s0 = d.seg_ptr[g], s1 = d.seg_ptr[g + 1];
    for (int c0 = 0; c0 < nc; c0 += 64) {
        const int c = c0 + lane;
        const bool valid = c < nc;
        const VT *col = vals + off + (valid ? c : 0);
        A a[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = 0;
        // 16 rows per batch; the last batch is clamped to row nr-1 and weighted
        // 0 past the end so that its loads are issued together
        for (int i = 0; i < nr; i += 16) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int r = i + q, rr = min(r, nr - 1);
                a[q] += (A)col[(int64_t)rr * nc] * (r < nr ? xs[rr] : A(0));
            }
        }
        A acc = 0;
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += a[q];
        if (valid) {
            int s = s0, sc = 0;
            while (s + 1 < s1 && c >= sc + d.seg_len[s]) sc += d.seg_len[s++];
            const int o = d.seg_in[s] + (c - sc);
            y[o] = (YT)((A)y[o] + acc);
        }
    }
}

// Transposes every group's panel in place of a second buffer: out holds P^T
// (ncols x nrows, row-major) at the group's offset.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose_panels(RowPanelDev d, const T *__restrict__ in,
                                                          T *__restrict__ out)
{
    const int g = blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    for (int e = threadIdx.x; e < nr * nc; e += 256) {
        const int r = e / nc, c = e % nc;
        out[off + (int64_t)c * nr + r] = in[off + e];
    }
}

// Transposed copy grouped by column: out group g collects the blocks of
// column panel group g; entry (i, j) of block b (row i of its row panel,
// column j of the segment) goes to row j, column c0(b) + i of group g.
template <typename T>
__global__ __launch_bounds__(256) void k_regroup_transpose(ColPanelDev cp, RowPanelDev out,
                                                           const T *__restrict__ in, T *__restrict__ o)
{
    const int g = blockIdx.x;
    const int nr = out.nrows[g], nc = out.ncols[g];
    const int64_t ooff = out.val_off[g];
    int c0 = 0;
    for (int b = cp.blk_ptr[g]; b < cp.blk_ptr[g + 1]; ++b) {
        const int nb = cp.b_nrows[b], stride = cp.b_stride[b];
        const int64_t ioff = cp.b_val_off[b] + cp.b_c0[b];
        for (int e = threadIdx.x; e < nb * nr; e += 256) {
            const int i = e / nr, j = e % nr;
            o[ooff + (int64_t)j * nc + c0 + i] = in[ioff + (int64_t)i * stride + j];
        }
        c0 += nb;
    }
}

template <typename VT, typename XT, typename YT>
void launch_colpanel(const ColPanels &cp, int g0, int g1, const VT *vals, const XT *x, YT *y,
                     hipStream_t st, Role role, bool accumulate)
{
    if (g1 <= g0) return;
    const int acc = accumulate ? 1 : 0;
    switch (role) {
    case Role::Leaf:
        hipLaunchKernelGGL((k_colpanel_narrow<VT, XT, YT, 0>), dim3(g1 - g0), dim3(64), 0, st, cp.dev, g0, vals, x,
                           y, acc);
        break;
    case Role::Transfer:
        hipLaunchKernelGGL((k_colpanel_narrow<VT, XT, YT, 1>), dim3(g1 - g0), dim3(64), 0, st, cp.dev, g0, vals, x,
                           y, acc);
        break;
    case Role::Coupling:
        hipLaunchKernelGGL((k_colpanel<VT, XT, YT, 2>), dim3(g1 - g0), dim3(NT), 0, st, cp.dev, g0, vals, x, y);
        break;
    default:
        hipLaunchKernelGGL((k_colpanel<VT, XT, YT, 3>), dim3(g1 - g0), dim3(NT), 0, st, cp.dev, g0, vals, x, y);
        break;
    }
    hip_check(hipGetLastError(), "column panel launch");
}

template <typename VT, typename XT, typename YT>
void launch_rowpanelT(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y, hipStream_t st,
                      Role role)
{
    if (g1 <= g0) return;
    using A = typename Acc<VT>::type;
    const size_t shm = sizeof(A) * (size_t)std::max(rp.max_nrows, 1);
    if (role == Role::Leaf)
        hipLaunchKernelGGL((k_rowpanelT_narrow<VT, XT, YT, 0>), dim3(g1 - g0), dim3(64), shm, st, rp.dev, g0, vals,
                           x, y);
    else
        hipLaunchKernelGGL((k_rowpanelT_narrow<VT, XT, YT, 1>), dim3(g1 - g0), dim3(64), shm, st, rp.dev, g0, vals,
                           x, y);
    hip_check(hipGetLastError(), "transposed row panel launch");
}

template <typename T>
void launch_regroup_transpose(const ColPanels &cp, const RowPanels &out, const T *in, T *o, hipStream_t st)
{
    if (cp.ngroups() != out.ngroups()) fail(H2B_EINVAL, "transposed copy does not match its column panels");
    if (out.ngroups() == 0) return;
    hipLaunchKernelGGL(k_regroup_transpose<T>, dim3(out.ngroups()), dim3(256), 0, st, cp.dev, out.dev, in, o);
    hip_check(hipGetLastError(), "transposed copy launch");
}

template <typename T> void launch_transpose_panels(const RowPanels &rp, const T *in, T *out, hipStream_t st)
{
    if (rp.ngroups() == 0) return;
    hipLaunchKernelGGL(k_transpose_panels<T>, dim3(rp.ngroups()), dim3(256), 0, st, rp.dev, in, out);
    hip_check(hipGetLastError(), "transpose launch");
}

void launch_gather(const int32_t *perm, int64_t n, int nrhs, const double *x, int64_t ldx,
                   double *xp, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(n * nrhs)), dim3(NT), 0, st, perm, n, nrhs, x, ldx, xp);
    hip_check(hipGetLastError(), "gather launch");
}

void launch_scatter_add(const int32_t *perm, int64_t n, int nrhs, double alpha, const double *yp,
                        const double *yp2, double *y, int64_t ldy, hipStream_t st)
{
    hipLaunchKernelGGL(k_scatter_add, dim3(blocks_for(n * nrhs)), dim3(NT), 0, st, perm, n, nrhs, alpha,
                       yp, yp2, y, ldy);
    hip_check(hipGetLastError(), "scatter launch");
}

template <typename T> void launch_fill_zero(T *p, int64_t n, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(blocks_for(n)), dim3(NT), 0, st, p, n);
    hip_check(hipGetLastError(), "fill launch");
}

// explicit instantiations
template void launch_leaf_basis<double>(bool, const RowPanels &, const int32_t *, const double *, int,
                                        const GeoDev &, const QuadDev &, double *, hipStream_t);
template void launch_leaf_basis<float>(bool, const RowPanels &, const int32_t *, const double *, int,
                                       const GeoDev &, const QuadDev &, float *, hipStream_t);
template void launch_transfer<double>(const RowPanels &, const double *, int, double *, hipStream_t);
template void launch_transfer<float>(const RowPanels &, const double *, int, float *, hipStream_t);
template void launch_coupling<double>(const RowPanels &, const double *, const double *, int, double *,
                                      hipStream_t);
template void launch_coupling<float>(const RowPanels &, const double *, const double *, int, float *,
                                     hipStream_t);
template void launch_coupling<bf16_t>(const RowPanels &, const double *, const double *, int, bf16_t *,
                                      hipStream_t);
template void launch_fill_zero<double>(double *, int64_t, hipStream_t);
template void launch_leaf_grad<double>(const RowPanels &, const int32_t *, const double *, int, const GeoDev &,
                                       const QuadDev &, const double *, const double *, const double *,
                                       const double *, double *, double *, double *, hipStream_t);
template void launch_leaf_grad<float>(const RowPanels &, const int32_t *, const double *, int, const GeoDev &,
                                      const QuadDev &, const float *, const float *, const double *,
                                      const double *, double *, double *, double *, hipStream_t);
template void launch_fill_zero<float>(float *, int64_t, hipStream_t);
template void launch_transpose_panels<double>(const RowPanels &, const double *, double *, hipStream_t);
template void launch_rowpanelT<double, double, double>(const RowPanels &, int, int, const double *,
                                                      const double *, double *, hipStream_t, Role);
template void launch_rowpanelT<float, float, float>(const RowPanels &, int, int, const float *, const float *,
                                                   float *, hipStream_t, Role);
template void launch_rowpanelT<float, float, double>(const RowPanels &, int, int, const float *, const float *,
                                                    double *, hipStream_t, Role);
template void launch_regroup_transpose<double>(const ColPanels &, const RowPanels &, const double *, double *,
                                               hipStream_t);
template void launch_regroup_transpose<float>(const ColPanels &, const RowPanels &, const float *, float *,
                                              hipStream_t);
template void launch_regroup_transpose<bf16_t>(const ColPanels &, const RowPanels &, const bf16_t *, bf16_t *,
                                               hipStream_t);
template void launch_transpose_panels<float>(const RowPanels &, const float *, float *, hipStream_t);
#define H2B_PANEL_INST(VT, XT, YT)                                                                      \
    template void launch_rowpanel<VT, XT, YT>(const RowPanels &, int, int, const VT *, const XT *, YT *, \
                                              bool, hipStream_t, Role);                                 \
    template void launch_colpanel<VT, XT, YT>(const ColPanels &, int, int, const VT *, const XT *, YT *, \
                                              hipStream_t, Role, bool);
H2B_PANEL_INST(double, double, double)
H2B_PANEL_INST(float, double, float)
H2B_PANEL_INST(float, float, float)
H2B_PANEL_INST(float, float, double)
H2B_PANEL_INST(bf16_t, float, float)
#undef H2B_PANEL_INST

}  // namespace h2b
