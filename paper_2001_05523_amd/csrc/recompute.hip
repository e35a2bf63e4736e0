// Coupling products with the coupling matrices evaluated on the fly.
//
// The coupling matrix of a farfield block is the kernel function at the two
// clusters' interpolation points, S_ts[nu, mu] = g(xi_{t,nu}, xi_{s,mu})
// (Section 2, eq. (vsw); Section 3), so it need not be stored: every product
// evaluates its k_t k_s entries again from the 3 m Chebyshev coordinates of t
// and s.  That trades the largest stored object for ALU work (one reciprocal
// square root and a few FMAs per entry) and makes orders whose coupling
// storage would not fit usable.
//
// With algebraic recompression the stored coupling would be P_t S_ts P_s^T,
// P_c = (new basis)^T (interpolation basis) of cluster c (k'_c x k).  The
// projections are applied once per cluster instead of once per block:
//   x~_s = P_s^T x^_s for every input cluster,
//   y~_t = sum_s S_ts x~_s over the farfield blocks (evaluated here),
//   y^_t += P_t y~_t for every output cluster.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "device.hpp"
#include "op.hpp"

namespace h2b {

namespace {

constexpr double INV_4PI = 0.0795774715459476678844418816862571810;  // 1 / (4 pi)

// One wave per group (output cluster t): lane l owns the rows nu = l + 64 j,
// j < NJ; the segments (farfield partners s) are walked in order with their
// point coordinates and inputs at wave-uniform addresses.
template <int NJ>
__global__ __launch_bounds__(64) void k_coupling_eval(RowPanelDev d, const double *__restrict__ gax,
                                                      const double *__restrict__ sax, int m,
                                                      const double *__restrict__ x, double *__restrict__ y)
{
    const int g = blockIdx.x;
    const int t = d.tag[g];
    const int k = d.nrows[g];
    const int64_t out = d.out_begin[g];
    const int lane = threadIdx.x;
    const double *pt = gax + (int64_t)t * 3 * m;
    double px[NJ], py[NJ], pz[NJ], acc[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int nu = min(lane + 64 * j, k - 1);
        px[j] = pt[nu % m];
        py[j] = pt[m + (nu / m) % m];
        pz[j] = pt[2 * m + nu / (m * m)];
        acc[j] = 0.0;
    }
    const int s0 = d.seg_ptr[g], s1 = d.seg_ptr[g + 1];
    for (int si = s0; si < s1; ++si) {
        const int s = d.seg_tag[si];
        const double *ps = sax + (int64_t)s * 3 * m;
        const double *xs = x + d.seg_in[si];
        int mu = 0;
        for (int m3 = 0; m3 < m; ++m3) {
            const double qz = ps[2 * m + m3];
            for (int m2 = 0; m2 < m; ++m2) {
                const double qy = ps[m + m2];
                double ryz[NJ];
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    const double dy = py[j] - qy, dz = pz[j] - qz;
                    ryz[j] = dy * dy + dz * dz;
                }
                for (int m1 = 0; m1 < m; ++m1, ++mu) {
                    const double xv = xs[mu];
                    const double qx = ps[m1];
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const double dx = px[j] - qx;
                        acc[j] += xv * rsqrt(dx * dx + ryz[j]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int nu = lane + 64 * j;
        if (nu < k) y[out + nu] += INV_4PI * acc[j];
    }
}

// Blocks of rb right-hand sides (vectors row-major, entry (i, r) at i rb + r):
// one workgroup of 256 threads per group.  For every 64-row slice of the
// output and 64-column slice of each partner's points, the 64 x 64 tile of
// S_ts is evaluated into LDS (transposed, so that a wave reads consecutive
// rows) beside the matching 64 x rb slice of the input, and every thread
// accumulates rb / 4 columns of one row.
constexpr int MT = 256;

__global__ __launch_bounds__(MT) void k_coupling_eval_mrhs(RowPanelDev d, const double *__restrict__ gax,
                                                           const double *__restrict__ sax, int m, int rb,
                                                           const double *__restrict__ x, double *__restrict__ y)
{
    __shared__ double St[64][65];   // St[mu][nu] of the current tile
    __shared__ double Xs[64][64];   // inputs of the tile: 64 points x rb columns
    const int g = blockIdx.x;
    const int t = d.tag[g];
    const int k = d.nrows[g];
    const int64_t out = d.out_begin[g];
    const int tid = threadIdx.x;
    const int row = tid & 63;              // row of the slice this thread accumulates
    const int cpt = rb / 4;                // columns per thread
    const int c0 = (tid >> 6) * cpt;       // its first column (uniform per wave)
    const double *pt = gax + (int64_t)t * 3 * m;
    const int s0 = d.seg_ptr[g], s1 = d.seg_ptr[g + 1];
    for (int r0 = 0; r0 < k; r0 += 64) {
        double acc[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = 0.0;
        for (int si = s0; si < s1; ++si) {
            const int s = d.seg_tag[si];
            const int ks = d.seg_len[si];
            const double *ps = sax + (int64_t)s * 3 * m;
            const int64_t in = d.seg_in[si];
            for (int q0 = 0; q0 < ks; q0 += 64) {
                __syncthreads();  // the previous tile has been read
                for (int e = tid; e < 64 * 64; e += MT) {
                    const int nu = r0 + (e & 63), mu = q0 + (e >> 6);
                    double v = 0.0;
                    if (nu < k && mu < ks) {
                        const double dx = pt[nu % m] - ps[mu % m];
                        const double dy = pt[m + (nu / m) % m] - ps[m + (mu / m) % m];
                        const double dz = pt[2 * m + nu / (m * m)] - ps[2 * m + mu / (m * m)];
                        v = rsqrt(dx * dx + dy * dy + dz * dz);
                    }
                    St[e >> 6][e & 63] = v;
                }
                const int nq = min(64, ks - q0);
                for (int e = tid; e < 64 * rb; e += MT) {
                    const int q = e / rb, c = e % rb;
                    Xs[q][c] = q < nq ? x[(in + q0 + q) * rb + c] : 0.0;
                }
                __syncthreads();
                for (int q = 0; q < nq; ++q) {
                    const double sv = St[q][row];
#pragma unroll
                    for (int c = 0; c < 16; ++c)
                        if (c < cpt) acc[c] += sv * Xs[q][c0 + c];
                }
            }
        }
        const int nu = r0 + row;
        if (nu < k)
#pragma unroll
            for (int c = 0; c < 16; ++c)
                if (c < cpt) y[(out + nu) * rb + c0 + c] += INV_4PI * acc[c];
    }
}

void launch_eval(const RowPanels &P, const double *gax, const double *sax, int m, int rb, const double *x,
                 double *y, hipStream_t st)
{
    if (P.ngroups() == 0) return;
    const int k = m * m * m;
    if (rb == 1) {
        const int nj = (k + 63) / 64;
        switch (nj) {
        case 1: hipLaunchKernelGGL(k_coupling_eval<1>, dim3(P.ngroups()), dim3(64), 0, st, P.dev, gax, sax, m, x, y); break;
        case 2: hipLaunchKernelGGL(k_coupling_eval<2>, dim3(P.ngroups()), dim3(64), 0, st, P.dev, gax, sax, m, x, y); break;
        case 3: hipLaunchKernelGGL(k_coupling_eval<3>, dim3(P.ngroups()), dim3(64), 0, st, P.dev, gax, sax, m, x, y); break;
        default: hipLaunchKernelGGL(k_coupling_eval<4>, dim3(P.ngroups()), dim3(64), 0, st, P.dev, gax, sax, m, x, y); break;
        }
    } else {
        if (rb != 16 && rb != 32 && rb != 64) fail(H2B_EINVAL, "block width must be 16, 32 or 64");
        hipLaunchKernelGGL(k_coupling_eval_mrhs, dim3(P.ngroups()), dim3(MT), 0, st, P.dev, gax, sax, m, rb, x, y);
    }
    hip_check(hipGetLastError(), "coupling evaluation launch");
}

}  // namespace

void setup_recompute(Op &op, hipStream_t st)
{
    // groups of the transposed product (by column cluster), structure only
    if (op.cpl_R.ngroups() == 0 && op.cpl_T.ngroups() > 0) {
        regroup_transposed(op.cpl_T, op.cpl_R);
        op.cpl_R.upload(st);
    }
    const int m = op.params.order_m;
    const int k = m * m * m;
    if (op.cpl.max_nrows > k || op.cpl_R.max_nrows > k)
        fail(H2B_EDEVICE, "coupling groups larger than the interpolation rank");
}

void set_projection(Basis &B, int k, const std::vector<std::vector<double>> &P, hipStream_t st)
{
    const Tree &T = *B.tree;
    B.proj = RowPanels();
    B.proj_T = ColPanels();
    std::vector<double> vals;
    for (int64_t c = 0; c < T.nclusters(); ++c) {
        if (B.rank[c] == 0) continue;
        B.proj.begin_group((int)c, (int)B.hat_off[c], B.rank[c]);
        B.proj.add_segment((int)(c * k), k, (int)c);
        B.proj.end_group();
        vals.insert(vals.end(), P[c].begin(), P[c].end());
    }
    if ((int64_t)vals.size() != B.proj.total) fail(H2B_EDEVICE, "projection sizes do not match the ranks");
    transpose_panels(B.proj, 0, B.proj.ngroups(), B.proj_T);
    B.proj.upload(st);
    B.proj_T.upload(st);
    B.proj_vals.alloc(sizeof(double) * std::max<size_t>(vals.size(), 1));
    hip_check(hipMemcpyAsync(B.proj_vals.p, vals.data(), sizeof(double) * vals.size(), hipMemcpyHostToDevice, st),
              "projection upload");
    hip_check(hipStreamSynchronize(st), "projection upload");
    B.has_proj = true;
}

void recompute_coupling(const Op &op, int trans, int rb, const double *xhat, double *yhat, double *xt, double *yt,
                        hipStream_t st)
{
    const Basis &Bin = trans ? *op.rowb : *op.colb;
    const Basis &Bout = trans ? *op.colb : *op.rowb;
    const RowPanels &P = trans ? op.cpl_R : op.cpl;
    const int m = op.params.order_m;
    const int k = m * m * m;
    if (!Bin.has_proj) {
        launch_eval(P, Bout.axes.as<double>(), Bin.axes.as<double>(), m, rb, xhat, yhat, st);
        return;
    }
    const int64_t nin = Bin.tree->nclusters() * (int64_t)k, nout = Bout.tree->nclusters() * (int64_t)k;
    launch_fill_zero<double>(xt, nin * rb, st);
    launch_fill_zero<double>(yt, nout * rb, st);
    if (rb == 1) {
        launch_colpanel<double, double, double>(Bin.proj_T, 0, Bin.proj_T.ngroups(), Bin.proj_vals.as<double>(),
                                                xhat, xt, st, Role::Transfer, true);
        launch_eval(P, Bout.axes.as<double>(), Bin.axes.as<double>(), m, 1, xt, yt, st);
        launch_rowpanel<double, double, double>(Bout.proj, 0, Bout.proj.ngroups(), Bout.proj_vals.as<double>(), yt,
                                                yhat, true, st, Role::Transfer);
    } else {
        launch_colpanel_mrhs<double, double, double>(Bin.proj_T, 0, Bin.proj_T.ngroups(), rb,
                                                     Bin.proj_vals.as<double>(), xhat, xt, true, st, Role::Transfer);
        launch_eval(P, Bout.axes.as<double>(), Bin.axes.as<double>(), m, rb, xt, yt, st);
        launch_rowpanel_mrhs<double, double, double>(Bout.proj, 0, Bout.proj.ngroups(), rb,
                                                     Bout.proj_vals.as<double>(), yt, yhat, true, st, Role::Transfer);
    }
}

}  // namespace h2b
