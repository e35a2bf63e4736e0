// Dirichlet-to-Neumann and Neumann-to-Dirichlet solves: the mixed mass matrix
// of Section 1, the hypersingular matrix W through its representation by the
// single-layer operator (W = sum_d C_d^T G C_d, C_d the d-th component of the
// surface curls of the hat functions, constant on each flat triangle), and
// the conjugate gradient method on the H^2 product of G or on W (eqs.
// (matrix_dtn), (matrix_ntd), solved by a Krylov method in the experiments
// of Section 5).
//
// Every scalar of the iteration (rho, alpha, beta, the count and the stop
// flag) lives in device memory, so the host only queues work: one iteration
// is the H^2 product q = A p followed by five small vector kernels, and a
// batch of check_every iterations is captured once into a HIP graph (each
// product with its nearfield and far field as parallel branches) and
// replayed.  Inner products are two-stage reductions over a fixed grid
// (partials per workgroup in a fixed slicing, then one workgroup sums them in
// index order), so the same input gives the same bits.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>

#include "hchol.hpp"
#include "op.hpp"

namespace h2b {

namespace {

constexpr int KT = 256;      // threads per workgroup of the vector kernels
constexpr int KMAXB = 1024;  // most partial sums of one reduction

// State of one solve in device memory.
struct CgState {
    double rho;      // r^T z of the current residual (z = r without a preconditioner)
    double rr;       // r^T r (the stopping test and the reported residual)
    double bnorm2;   // b^T b
    double thresh2;  // (tol ||b||)^2
    double alpha, beta;
    int iter;        // iterations done
    int status;      // 0 running, else h2b_cg_status
    int max_iter;
    int pad;
    double shift;    // hypersingular form: coefficient of w1 removed from b, then of 1 removed from x
};

__device__ inline double wave_total(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum of v over the workgroup in a fixed order, valid in thread 0.
__device__ inline double group_total(double v, double *lds)
{
    v = wave_total(v);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < KT / 64; ++w) s += lds[w];
    __syncthreads();
    return s;
}

// Sum of part[0..nb) in index order per thread slice, valid in thread 0.
__device__ inline double parts_total(const double *part, int nb, double *lds)
{
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += KT) acc += part[i];
    return group_total(acc, lds);
}

__device__ inline double rel_norm(double rr, double bb) { return sqrt(bb > 0.0 ? rr / bb : rr); }

// part[g] = sum of a_i c_i (c = NULL: of a_i) over the slice of workgroup g.
__global__ __launch_bounds__(KT) void k_dot_part(const double *__restrict__ a, const double *__restrict__ c,
                                                 int64_t n, double *__restrict__ part)
{
    __shared__ double lds[KT / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        acc += c ? a[i] * c[i] : a[i];
    const double s = group_total(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(KT) void k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) dst[i] = src[i];
}

// Initial state from the partial sums of b^T b, r0^T r0 and (preconditioned)
// r0^T z0 (prz = NULL: z0 = r0).
__global__ __launch_bounds__(KT) void k_cg_start(const double *__restrict__ pb, const double *__restrict__ pr,
                                                 const double *__restrict__ prz, int nb, double tol, int max_iter,
                                                 CgState *S, double *hist)
{
    __shared__ double lds[KT / 64];
    const double bb = parts_total(pb, nb, lds);
    const double rr = parts_total(pr, nb, lds);
    const double rz = prz ? parts_total(prz, nb, lds) : rr;
    if (threadIdx.x == 0) {
        S->bnorm2 = bb;
        S->thresh2 = tol * tol * bb;
        S->rho = rz;
        S->rr = rr;
        S->alpha = 0.0;
        S->beta = 0.0;
        S->iter = 0;
        S->max_iter = max_iter;
        S->status = rr <= tol * tol * bb ? H2B_CG_CONVERGED : max_iter == 0 ? H2B_CG_MAXITER : 0;
        hist[0] = rel_norm(rr, bb);
    }
}

// S->shift = (sum of pnum) / (sum of pden).
__global__ __launch_bounds__(KT) void k_ratio(const double *__restrict__ pnum, const double *__restrict__ pden,
                                              int nb, CgState *S)
{
    __shared__ double lds[KT / 64];
    const double num = parts_total(pnum, nb, lds);
    const double den = parts_total(pden, nb, lds);
    if (threadIdx.x == 0) S->shift = den != 0.0 ? num / den : 0.0;
}

// y = a - S->shift * w (w = NULL: the vector of ones).
__global__ __launch_bounds__(KT) void k_sub_shift(const double *a, const double *__restrict__ w, int64_t n,
                                                  const CgState *S, double *y)
{
    const double c = S->shift;
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        y[i] = a[i] - c * (w ? w[i] : 1.0);
}

// *out = sum of part[0..nb) (the second stage of a dot product).
__global__ __launch_bounds__(KT) void k_parts_to(const double *__restrict__ part, int nb, double *__restrict__ out)
{
    __shared__ double lds[KT / 64];
    const double s = parts_total(part, nb, lds);
    if (threadIdx.x == 0) *out = s;
}

// alpha = rho / p^T q (0 once stopped; breakdown when p^T q is not positive).
__global__ __launch_bounds__(KT) void k_cg_alpha(const double *__restrict__ part, int nb, CgState *S)
{
    __shared__ double lds[KT / 64];
    const double pq = parts_total(part, nb, lds);
    if (threadIdx.x == 0) {
        double a = 0.0;
        if (S->status == 0) {
            if (pq > 0.0 && isfinite(pq))
                a = S->rho / pq;
            else
                S->status = H2B_CG_BREAKDOWN;
        }
        S->alpha = a;
    }
}

// x += alpha p, r -= alpha q, q = 0 for the next product (which accumulates
// into it), part[g] = slice sum of r_i^2.
__global__ __launch_bounds__(KT) void k_cg_step(double *__restrict__ x, double *__restrict__ r,
                                                const double *__restrict__ p, double *__restrict__ q, int64_t n,
                                                const CgState *S, double *__restrict__ part)
{
    __shared__ double lds[KT / 64];
    const double a = S->alpha;
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) {
        double ri = r[i];
        if (a != 0.0) {
            ri -= a * q[i];
            x[i] += a * p[i];
            r[i] = ri;
        }
        q[i] = 0.0;
        acc += ri * ri;
    }
    const double s = group_total(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// rr' = r^T r, rho' = r^T z (prz = NULL: rho' = rr'), beta = rho' / rho,
// count the iteration and test the stop on rr'.
__global__ __launch_bounds__(KT) void k_cg_beta(const double *__restrict__ part, const double *__restrict__ prz,
                                                int nb, CgState *S, double *hist)
{
    __shared__ double lds[KT / 64];
    const double rr = parts_total(part, nb, lds);
    const double rz = prz ? parts_total(prz, nb, lds) : rr;
    if (threadIdx.x == 0) {
        double b = 0.0;
        if (S->status == 0) {
            const int it = S->iter + 1;
            b = rz / S->rho;
            S->rho = rz;
            S->rr = rr;
            S->iter = it;
            hist[it] = rel_norm(rr, S->bnorm2);
            if (rr <= S->thresh2)
                S->status = H2B_CG_CONVERGED;
            else if (it >= S->max_iter)
                S->status = H2B_CG_MAXITER;
        }
        S->beta = b;
    }
}

// p = z + beta p (z = r without a preconditioner).
__global__ __launch_bounds__(KT) void k_cg_direction(double *__restrict__ p, const double *__restrict__ r, int64_t n,
                                                     const CgState *S)
{
    const double b = S->beta;
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        p[i] = r[i] + b * p[i];
}

__device__ inline double tri_area(const GeoDev &g, int64_t i)
{
    const int a = g.t0[i], b = g.t1[i], c = g.t2[i];
    const double ux = g.vx[b] - g.vx[a], uy = g.vy[b] - g.vy[a], uz = g.vz[b] - g.vz[a];
    const double wx = g.vx[c] - g.vx[a], wy = g.vy[c] - g.vy[a], wz = g.vz[c] - g.vz[a];
    const double cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
    return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
}

// y_i += alpha |tau_i| / 3 (x_a + x_b + x_c) over the corners of tau_i.
__global__ __launch_bounds__(KT) void k_mass(GeoDev g, int64_t nt, double alpha, const double *__restrict__ x,
                                             double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < nt; i += (int64_t)gridDim.x * KT)
        y[i] += alpha * (tri_area(g, i) / 3.0) * (x[g.t0[i]] + x[g.t1[i]] + x[g.t2[i]]);
}

// y_j += alpha sum over the triangles tau around vertex j of |tau| / 3 x_tau.
__global__ __launch_bounds__(KT) void k_mass_t(GeoDev g, int64_t nv, double alpha, const double *__restrict__ x,
                                               double *__restrict__ y)
{
    for (int64_t j = blockIdx.x * (int64_t)KT + threadIdx.x; j < nv; j += (int64_t)gridDim.x * KT) {
        double s = 0.0;
        for (int64_t e = g.vt_ptr[j]; e < g.vt_ptr[j + 1]; ++e) {
            const int32_t t = g.vt_idx[e];
            s += (tri_area(g, t) / 3.0) * x[t];
        }
        y[j] += alpha * s;
    }
}

// w1_j = int phi_j = sum over the triangles t around vertex j of |t| / 3.
__global__ __launch_bounds__(KT) void k_p1_integrals(GeoDev g, int64_t nv, double *__restrict__ w1)
{
    for (int64_t j = blockIdx.x * (int64_t)KT + threadIdx.x; j < nv; j += (int64_t)gridDim.x * KT) {
        double s = 0.0;
        for (int64_t e = g.vt_ptr[j]; e < g.vt_ptr[j + 1]; ++e) s += tri_area(g, g.vt_idx[e]) / 3.0;
        w1[j] = s;
    }
}

// Surface curl of the hat function of corner j on triangle t: with the
// corners (a, b, c) counter-clockwise, curl phi_a = (x_b - x_c) / (2|t|) and
// cyclically (n x grad phi_a, n the outward normal).
__device__ inline void corner_curl(const GeoDev &g, int32_t nxt, int32_t prv, double inv2a, double &cx, double &cy,
                                   double &cz)
{
    cx = (g.vx[nxt] - g.vx[prv]) * inv2a;
    cy = (g.vy[nxt] - g.vy[prv]) * inv2a;
    cz = (g.vz[nxt] - g.vz[prv]) * inv2a;
}

// c[t + d nt] = (C_d x)_t = sum over the corners j of t of x_j (curl phi_j)_d.
__global__ __launch_bounds__(KT) void k_curl(GeoDev g, int64_t nt, const double *__restrict__ x,
                                             double *__restrict__ c)
{
    for (int64_t t = blockIdx.x * (int64_t)KT + threadIdx.x; t < nt; t += (int64_t)gridDim.x * KT) {
        const int32_t a = g.t0[t], b = g.t1[t], d = g.t2[t];
        const double inv2a = 1.0 / (2.0 * tri_area(g, t));
        double sx = 0.0, sy = 0.0, sz = 0.0, cx, cy, cz;
        corner_curl(g, b, d, inv2a, cx, cy, cz);
        sx += x[a] * cx, sy += x[a] * cy, sz += x[a] * cz;
        corner_curl(g, d, a, inv2a, cx, cy, cz);
        sx += x[b] * cx, sy += x[b] * cy, sz += x[b] * cz;
        corner_curl(g, a, b, inv2a, cx, cy, cz);
        sx += x[d] * cx, sy += x[d] * cy, sz += x[d] * cz;
        c[t] = sx;
        c[t + nt] = sy;
        c[t + 2 * nt] = sz;
    }
}

// The transpose of k_curl in two passes.  First, per triangle t, the three
// corner contributions ct[3 t + c] = sum_d (curl phi_corner c on t)_d gc[t + d nt]
// (one area per triangle, coalesced); then, per vertex j,
// y_j += alpha sum over the triangles t around j of ct[3 t + (corner of j in t)].
__global__ __launch_bounds__(KT) void k_curl_corners(GeoDev g, int64_t nt, const double *__restrict__ gc,
                                                     double *__restrict__ ct)
{
    for (int64_t t = blockIdx.x * (int64_t)KT + threadIdx.x; t < nt; t += (int64_t)gridDim.x * KT) {
        const int32_t a = g.t0[t], b = g.t1[t], d = g.t2[t];
        const double inv2a = 1.0 / (2.0 * tri_area(g, t));
        const double gx = gc[t], gy = gc[t + nt], gz = gc[t + 2 * nt];
        double cx, cy, cz;
        corner_curl(g, b, d, inv2a, cx, cy, cz);
        ct[3 * t] = cx * gx + cy * gy + cz * gz;
        corner_curl(g, d, a, inv2a, cx, cy, cz);
        ct[3 * t + 1] = cx * gx + cy * gy + cz * gz;
        corner_curl(g, a, b, inv2a, cx, cy, cz);
        ct[3 * t + 2] = cx * gx + cy * gy + cz * gz;
    }
}

__global__ __launch_bounds__(KT) void k_curl_t(GeoDev g, int64_t nv, const double *__restrict__ ct, double alpha,
                                               double *__restrict__ y)
{
    for (int64_t j = blockIdx.x * (int64_t)KT + threadIdx.x; j < nv; j += (int64_t)gridDim.x * KT) {
        double s = 0.0;
        for (int64_t e = g.vt_ptr[j]; e < g.vt_ptr[j + 1]; ++e) {
            const int32_t t = g.vt_idx[e];
            const int corner = j == g.t0[t] ? 0 : j == g.t1[t] ? 1 : 2;
            s += ct[3 * (int64_t)t + corner];
        }
        y[j] += alpha * s;
    }
}

// Block-Jacobi preconditioner: the inverse of the symmetric part of every
// diagonal nearfield block N_tt (leaves of at most 64), by Gauss-Jordan
// elimination in LDS (no pivoting: the blocks of G are symmetric positive
// definite).  One workgroup per leaf.
__global__ __launch_bounds__(KT) void k_bj_invert(const int64_t *__restrict__ src, const int32_t *__restrict__ stride,
                                                  const int32_t *__restrict__ nn, const int64_t *__restrict__ dst,
                                                  const double *__restrict__ near, double *__restrict__ inv)
{
    __shared__ double A[64][65];
    __shared__ double fcol[64];
    __shared__ double piv;
    const int leaf = blockIdx.x, n = nn[leaf], ld = stride[leaf];
    const int64_t s0 = src[leaf];
    for (int e = threadIdx.x; e < n * n; e += KT) {
        const int i = e / n, j = e % n;
        A[i][j] = 0.5 * (near[s0 + (int64_t)i * ld + j] + near[s0 + (int64_t)j * ld + i]);
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (threadIdx.x == 0) piv = 1.0 / A[k][k];
        __syncthreads();
        for (int j = threadIdx.x; j < n; j += KT) A[k][j] = j == k ? piv : A[k][j] * piv;
        for (int i = threadIdx.x; i < n; i += KT) fcol[i] = i == k ? 0.0 : A[i][k];
        __syncthreads();
        for (int e = threadIdx.x; e < n * n; e += KT) {
            const int i = e / n, j = e % n;
            if (i == k) continue;
            A[i][j] = j == k ? -fcol[i] * A[k][k] : A[i][j] - fcol[i] * A[k][j];
        }
        __syncthreads();
    }
    const int64_t d0 = dst[leaf];
    for (int e = threadIdx.x; e < n * n; e += KT) inv[d0 + e] = A[e / n][e % n];
}

// z|_t = inv_t r|_t for every leaf t (positions begin..begin+n of the
// cluster order, original indices through perm); a wave per row, lanes
// over the columns.
__global__ __launch_bounds__(KT) void k_bj_apply(const int32_t *__restrict__ begin, const int32_t *__restrict__ nn,
                                                 const int64_t *__restrict__ dst, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ inv, const double *__restrict__ r,
                                                 double *__restrict__ z)
{
    __shared__ double rl[64];
    const int leaf = blockIdx.x, n = nn[leaf], b = begin[leaf];
    const int64_t d0 = dst[leaf];
    if (threadIdx.x < n) rl[threadIdx.x] = r[perm[b + threadIdx.x]];
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = w; i < n; i += KT / 64) {
        double v = lane < n ? inv[d0 + (int64_t)i * n + lane] * rl[lane] : 0.0;
        v = wave_total(v);
        if (lane == 0) z[perm[b + i]] = v;
    }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(KMAXB, (n + KT * 4 - 1) / (KT * 4))); }

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

// Owner of the resources of one solve.
struct CgRun {
    DevMem r, p, q, part, part2, state, hist, w1, bp, z, part3;
    CgState *host = nullptr;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~CgRun()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (host) (void)hipHostFree(host);
    }
};

}  // namespace

void mass_matvec(Op &op, int trans, double alpha, const double *x, double *y, hipStream_t st)
{
    const Mesh &M = *op.blocks->rows->mesh;
    const int64_t nin = trans ? M.nt : M.nv, nout = trans ? M.nv : M.nt;
    if (!x || !y) fail(H2B_EINVAL, "x and y must not be NULL");
    if (overlaps(x, sizeof(double) * nin, y, sizeof(double) * nout)) fail(H2B_EINVAL, "x and y overlap");
    if (nout == 0) return;
    if (trans)
        hipLaunchKernelGGL(k_mass_t, dim3(grid_for(nout)), dim3(KT), 0, st, op.geo, nout, alpha, x, y);
    else
        hipLaunchKernelGGL(k_mass, dim3(grid_for(nout)), dim3(KT), 0, st, op.geo, nout, alpha, x, y);
    hip_check(hipGetLastError(), "mass launch");
}

// Inverse diagonal blocks of the nearfield, once per operator.
static void prepare_block_jacobi(Op &A, hipStream_t st)
{
    if (A.bj_leaves > 0) return;
    if (A.kernel != H2B_SLP || A.blocks->rows != A.blocks->cols)
        fail(H2B_ENOTSUP, "the block-Jacobi preconditioner needs the single-layer operator on one tree");
    if (A.near.max_nrows > 64) fail(H2B_ENOTSUP, "the block-Jacobi preconditioner needs leaves of at most 64");
    const RowPanels &N = A.near;
    std::vector<int64_t> src, dst;
    std::vector<int32_t> stride, nn, begin;
    int64_t tot = 0;
    for (int g = 0; g < N.ngroups(); ++g) {
        const int t = N.group_tag[g];
        int seg = -1;
        for (int q = N.seg_ptr[g]; q < N.seg_ptr[g + 1]; ++q)
            if (N.seg_tag[q] == t) seg = q;
        if (seg < 0) fail(H2B_EDEVICE, "a leaf without its diagonal nearfield block");
        src.push_back(N.val_off[g] + N.seg_c0[seg]);
        stride.push_back(N.ncols[g]);
        nn.push_back(N.nrows[g]);
        begin.push_back(N.out_begin[g]);
        dst.push_back(tot);
        tot += (int64_t)N.nrows[g] * N.nrows[g];
    }
    Packer pk;
    const int64_t *d_src = nullptr;
    const int32_t *d_stride = nullptr;
    pk.add(src, const_cast<int64_t **>(&d_src));
    pk.add(dst, const_cast<int64_t **>(&A.bj_dst));
    pk.add(stride, const_cast<int32_t **>(&d_stride));
    pk.add(nn, const_cast<int32_t **>(&A.bj_n));
    pk.add(begin, const_cast<int32_t **>(&A.bj_begin));
    pk.upload(A.bj_mem, st);
    A.bj_inv.alloc(sizeof(double) * std::max<int64_t>(tot, 1));
    hipLaunchKernelGGL(k_bj_invert, dim3(N.ngroups()), dim3(KT), 0, st, d_src, d_stride, A.bj_n, A.bj_dst,
                       A.near_vals.as<double>(), A.bj_inv.as<double>());
    hip_check(hipGetLastError(), "block-Jacobi setup");
    hip_check(hipStreamSynchronize(st), "block-Jacobi setup");
    A.bj_leaves = N.ngroups();
}

static void check_single_layer(const Op &G)
{
    if (G.kernel != H2B_SLP || G.nrows != G.ncols)
        fail(H2B_EINVAL, "the hypersingular product needs the single-layer operator G");
}

void prepare_hypersingular(Op &G)
{
    check_single_layer(G);
    const size_t bytes = sizeof(double) * 3 * (size_t)G.nrows;
    if (G.hs_c.bytes < bytes) {
        G.hs_c.alloc(bytes);
        G.hs_g.alloc(bytes);
    }
}

void hypersingular_matvec(Op &G, double alpha, const double *x, double *y, hipStream_t st)
{
    check_single_layer(G);
    const Mesh &M = *G.blocks->rows->mesh;
    const int64_t nt = M.nt, nv = M.nv;
    if (!x || !y) fail(H2B_EINVAL, "x and y must not be NULL");
    if (overlaps(x, sizeof(double) * nv, y, sizeof(double) * nv)) fail(H2B_EINVAL, "x and y overlap");
    prepare_hypersingular(G);
    double *c = G.hs_c.as<double>(), *gc = G.hs_g.as<double>();
    hipLaunchKernelGGL(k_curl, dim3(grid_for(nt)), dim3(KT), 0, st, G.geo, nt, x, c);
    hip_check(hipGetLastError(), "curl launch");
    launch_fill_zero<double>(gc, 3 * nt, st);
    // three single-vector products: each reads G's storage at the HBM rate of
    // the row-panel kernels, while one three-column block product pads to the
    // 16-column matrix-core tiles (13.1 ms against 3 x 2.6 ms at 2M triangles)
    for (int d = 0; d < 3; ++d) matvec(G, 0, 1.0, c + d * nt, nt, gc + d * nt, nt, 1, st);
    // the curls are consumed by now: their buffer takes the corner contributions
    hipLaunchKernelGGL(k_curl_corners, dim3(grid_for(nt)), dim3(KT), 0, st, G.geo, nt, gc, c);
    hipLaunchKernelGGL(k_curl_t, dim3(grid_for(nv)), dim3(KT), 0, st, G.geo, nv, c, alpha, y);
    hip_check(hipGetLastError(), "curl transpose launch");
}

void slp_bilinear(Op &G, const double *x, const double *y, double *gy, double *out, hipStream_t st)
{
    if (G.kernel != H2B_SLP) fail(H2B_EINVAL, "the bilinear form needs the single-layer operator G");
    if (!x || !y || !gy || !out) fail(H2B_EINVAL, "NULL vector");
    const int64_t n = G.nrows;
    if (overlaps(gy, sizeof(double) * n, x, sizeof(double) * n) || overlaps(out, sizeof(double), gy, sizeof(double) * n) ||
        overlaps(out, sizeof(double), x, sizeof(double) * n))
        fail(H2B_EINVAL, "gy must not overlap x, and out none of x and gy");
    check_product_args(G, 0, y, n, gy, n, 1);
    launch_fill_zero<double>(gy, n, st);
    matvec(G, 0, 1.0, y, n, gy, n, 1, st);
    // the product has ended on st (its nearfield branch is joined before its
    // last kernel), so its permuted-input vector holds the partial sums
    const int nb = grid_for(n);
    double *part = G.xp.as<double>();
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, x, gy, n, part);
    hipLaunchKernelGGL(k_parts_to, dim3(1), dim3(KT), 0, st, part, nb, out);
    hip_check(hipGetLastError(), "bilinear form launch");
}

void cg_solve(Op &A, const double *b, double *x, const h2b_cg_params &prm, h2b_cg_result &res, double *history,
              hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    const bool hyp = prm.form == H2B_FORM_HYPERSINGULAR;
    if (prm.form != H2B_FORM_PRODUCT && !hyp) fail(H2B_EINVAL, "unknown operator form");
    if (prm.precond != H2B_PRECOND_NONE && prm.precond != H2B_PRECOND_BLOCK_JACOBI &&
        prm.precond != H2B_PRECOND_HCHOL)
        fail(H2B_EINVAL, "unknown preconditioner");
    const bool hc = prm.precond == H2B_PRECOND_HCHOL;
    const bool pc = prm.precond != H2B_PRECOND_NONE;
    if (pc && hyp) fail(H2B_ENOTSUP, "the preconditioners are built for the product form");
    if (hc && (!prm.hchol || !prm.hchol->p)) fail(H2B_EINVAL, "H2B_PRECOND_HCHOL needs the factor (params.hchol)");
    if (hyp) check_single_layer(A);
    if (!hyp && A.nrows != A.ncols) fail(H2B_EINVAL, "conjugate gradients need a square operator");
    const int64_t n = hyp ? A.blocks->rows->mesh->nv : A.nrows;
    // q += A p (or W p)
    auto apply = [&](const double *in, double *out, double alpha, hipStream_t s) {
        if (hyp)
            hypersingular_matvec(A, alpha, in, out, s);
        else
            matvec(A, 0, alpha, in, n, out, n, 1, s);
    };
    if (!b || !x) fail(H2B_EINVAL, "b and x must not be NULL");
    if (overlaps(b, sizeof(double) * n, x, sizeof(double) * n)) fail(H2B_EINVAL, "b and x overlap");
    if (!(prm.tol >= 0.0) || !std::isfinite(prm.tol)) fail(H2B_EINVAL, "tol must be finite and >= 0");
    if (prm.max_iter < 0) fail(H2B_EINVAL, "max_iter must be >= 0");
    if (prm.check_every < 1) fail(H2B_EINVAL, "check_every must be >= 1");
    if (hyp)
        prepare_hypersingular(A);
    else
        prepare_product(A, 1);
    if (hc) {
        if (prm.hchol->p->H->tree->n != n) fail(H2B_EINVAL, "the H-Cholesky factor has another size");
        if (!prm.hchol->p->uploaded) hchol_upload(*prm.hchol->p, st);
    } else if (pc) {
        prepare_block_jacobi(A, st);
    }

    CgRun w;
    const int nb = grid_for(n);
    w.r.alloc(sizeof(double) * n);
    w.p.alloc(sizeof(double) * n);
    w.q.alloc(sizeof(double) * n);
    w.part.alloc(sizeof(double) * KMAXB);
    w.part2.alloc(sizeof(double) * KMAXB);
    w.state.alloc(sizeof(CgState));
    w.hist.alloc(sizeof(double) * ((size_t)prm.max_iter + 1));
    hip_check(hipHostMalloc(reinterpret_cast<void **>(&w.host), sizeof(CgState), hipHostMallocDefault),
              "pinned state");
    if (pc) {
        w.z.alloc(sizeof(double) * n);
        w.part3.alloc(sizeof(double) * KMAXB);
    }
    double *z = pc ? w.z.as<double>() : nullptr, *part3 = pc ? w.part3.as<double>() : nullptr;
    // z = P r: block Jacobi over the leaves of the operator's row tree, or
    // the substitutions with the H-Cholesky factor
    auto precondition = [&](hipStream_t s) {
        if (hc)
            hchol_apply(*prm.hchol->p, w.r.as<double>(), z, s);
        else
            hipLaunchKernelGGL(k_bj_apply, dim3(A.bj_leaves), dim3(KT), 0, s, A.bj_begin, A.bj_n, A.bj_dst,
                               A.rowb->perm_dev, A.bj_inv.as<double>(), w.r.as<double>(), z);
        hipLaunchKernelGGL(k_dot_part, dim3(grid_for(n)), dim3(KT), 0, s, w.r.as<double>(), z, n, part3);
    };
    double *r = w.r.as<double>(), *p = w.p.as<double>(), *q = w.q.as<double>();
    double *part = w.part.as<double>(), *part2 = w.part2.as<double>(), *hist = w.hist.as<double>();
    CgState *S = w.state.as<CgState>();

    if (hyp) {
        // W annihilates constants and b is orthogonal to them only up to
        // quadrature error: solve W x = b - c w1 with c = 1^T b / 1^T w1
        // (w1_j = int phi_j), the consistent system whose solution with
        // int u_h = w1^T x = 0 is that of the system bordered by w1
        w.w1.alloc(sizeof(double) * n);
        w.bp.alloc(sizeof(double) * n);
        hipLaunchKernelGGL(k_p1_integrals, dim3(nb), dim3(KT), 0, st, A.geo, n, w.w1.as<double>());
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, b, nullptr, n, part);
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, w.w1.as<double>(), nullptr, n, part2);
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(KT), 0, st, part, part2, nb, S);
        hipLaunchKernelGGL(k_sub_shift, dim3(nb), dim3(KT), 0, st, b, w.w1.as<double>(), n, S, w.bp.as<double>());
        hip_check(hipGetLastError(), "cg projection");
        b = w.bp.as<double>();
    }
    // r0 = b - A x0, p0 = r0, q = 0
    if (prm.zero_guess) launch_fill_zero<double>(x, n, st);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(KT), 0, st, b, r, n);
    if (!prm.zero_guess) apply(x, r, -1.0, st);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, b, b, n, part);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, r, r, n, part2);
    if (pc) precondition(st);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(KT), 0, st, part, part2, part3, nb, prm.tol, prm.max_iter, S,
                       hist);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(KT), 0, st, pc ? z : r, p, n);
    launch_fill_zero<double>(q, n, st);
    hip_check(hipGetLastError(), "cg start");

    // the vector work of one iteration after q = A p
    auto update = [&](hipStream_t s) {
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, s, p, q, n, part);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(KT), 0, s, part, nb, S);
        hipLaunchKernelGGL(k_cg_step, dim3(nb), dim3(KT), 0, s, x, r, p, q, n, S, part2);
        if (pc) precondition(s);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(KT), 0, s, part2, part3, nb, S, hist);
        hipLaunchKernelGGL(k_cg_direction, dim3(nb), dim3(KT), 0, s, p, pc ? z : r, n, S);
        hip_check(hipGetLastError(), "cg iteration");
    };
    auto read_state = [&] {
        hip_check(hipMemcpyAsync(w.host, S, sizeof(CgState), hipMemcpyDeviceToHost, st), "state read");
        hip_check(hipStreamSynchronize(st), "state read");
        return *w.host;
    };

    const int per = prm.check_every;
    CgState cur = read_state();
    if (cur.status == 0 && prm.use_graph) {
        // one graph of `per` iterations, captured on a private stream (the
        // caller's stream may be the null stream, which cannot be captured);
        // inside it every product runs its nearfield and far field as
        // parallel branches
        hip_check(hipStreamCreateWithFlags(&w.cap, hipStreamNonBlocking), "stream create");
        hip_check(hipStreamBeginCapture(w.cap, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
            for (int k = 0; k < per; ++k) {
                apply(p, q, 1.0, w.cap);
                update(w.cap);
            }
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(w.cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(w.cap, &w.graph), "end capture");
        hip_check(hipGraphInstantiate(&w.exec, w.graph, nullptr, nullptr, 0), "graph instantiate");
    }
    // every batch but a stopped one advances the count by `per`, so this bound
    // is only a guard against a state that never stops
    const int64_t max_batches = (int64_t)prm.max_iter / per + 2;
    for (int64_t batch = 0; cur.status == 0 && batch < max_batches; ++batch) {
        if (w.exec)
            hip_check(hipGraphLaunch(w.exec, st), "graph launch");
        else
            for (int k = 0; k < per; ++k) {
                apply(p, q, 1.0, st);
                update(st);
            }
        cur = read_state();
    }
    if (cur.status == 0) fail(H2B_EDEVICE, "conjugate gradients did not reach a stop state");
    if (hyp) {
        // the representative with int u_h = w1^T x = 0
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, w.w1.as<double>(), x, n, part);
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, w.w1.as<double>(), nullptr, n, part2);
        hipLaunchKernelGGL(k_ratio, dim3(1), dim3(KT), 0, st, part, part2, nb, S);
        hipLaunchKernelGGL(k_sub_shift, dim3(nb), dim3(KT), 0, st, x, nullptr, n, S, x);
        hip_check(hipGetLastError(), "cg normalisation");
        hip_check(hipStreamSynchronize(st), "cg normalisation");
    }
    if (history)
        hip_check(hipMemcpy(history, hist, sizeof(double) * ((size_t)cur.iter + 1), hipMemcpyDeviceToHost),
                  "history read");
    res.iterations = cur.iter;
    res.status = cur.status;
    res.rel_residual = sqrt(cur.bnorm2 > 0.0 ? cur.rr / cur.bnorm2 : cur.rr);
    res.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace h2b
