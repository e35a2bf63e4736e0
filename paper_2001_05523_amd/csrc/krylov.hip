// Dirichlet-to-Neumann solve: the mixed mass matrix of Section 1 and the
// conjugate gradient method on the H^2 product (eq. (matrix_dtn), solved by a
// Krylov method in the experiments of Section 5).
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

#include "op.hpp"

namespace h2b {

namespace {

constexpr int KT = 256;      // threads per workgroup of the vector kernels
constexpr int KMAXB = 1024;  // most partial sums of one reduction

// State of one solve in device memory.
struct CgState {
    double rho;      // r^T r of the current residual
    double bnorm2;   // b^T b
    double thresh2;  // (tol ||b||)^2
    double alpha, beta;
    int iter;        // iterations done
    int status;      // 0 running, else h2b_cg_status
    int max_iter;
    int pad;
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

// part[g] = sum of a_i c_i over the slice of workgroup g.
__global__ __launch_bounds__(KT) void k_dot_part(const double *__restrict__ a, const double *__restrict__ c,
                                                 int64_t n, double *__restrict__ part)
{
    __shared__ double lds[KT / 64];
    double acc = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT)
        acc += a[i] * c[i];
    const double s = group_total(acc, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(KT) void k_copy(const double *__restrict__ src, double *__restrict__ dst, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)KT + threadIdx.x; i < n; i += (int64_t)gridDim.x * KT) dst[i] = src[i];
}

// Initial state from the partial sums of b^T b and r0^T r0.
__global__ __launch_bounds__(KT) void k_cg_start(const double *__restrict__ pb, const double *__restrict__ pr,
                                                 int nb, double tol, int max_iter, CgState *S, double *hist)
{
    __shared__ double lds[KT / 64];
    const double bb = parts_total(pb, nb, lds);
    const double rr = parts_total(pr, nb, lds);
    if (threadIdx.x == 0) {
        S->bnorm2 = bb;
        S->thresh2 = tol * tol * bb;
        S->rho = rr;
        S->alpha = 0.0;
        S->beta = 0.0;
        S->iter = 0;
        S->max_iter = max_iter;
        S->status = rr <= tol * tol * bb ? H2B_CG_CONVERGED : max_iter == 0 ? H2B_CG_MAXITER : 0;
        hist[0] = rel_norm(rr, bb);
    }
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

// rho' = r^T r, beta = rho' / rho, count the iteration and test the stop.
__global__ __launch_bounds__(KT) void k_cg_beta(const double *__restrict__ part, int nb, CgState *S, double *hist)
{
    __shared__ double lds[KT / 64];
    const double rr = parts_total(part, nb, lds);
    if (threadIdx.x == 0) {
        double b = 0.0;
        if (S->status == 0) {
            const int it = S->iter + 1;
            b = rr / S->rho;
            S->rho = rr;
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

// p = r + beta p.
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

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(KMAXB, (n + KT * 4 - 1) / (KT * 4))); }

bool overlaps(const void *a, size_t na, const void *b, size_t nb)
{
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + nb && y < x + na;
}

// Owner of the resources of one solve.
struct CgRun {
    DevMem r, p, q, part, part2, state, hist;
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

void cg_solve(Op &A, const double *b, double *x, const h2b_cg_params &prm, h2b_cg_result &res, double *history,
              hipStream_t st)
{
    const auto t0 = std::chrono::steady_clock::now();
    if (A.nrows != A.ncols) fail(H2B_EINVAL, "conjugate gradients need a square operator");
    const int64_t n = A.nrows;
    if (!b || !x) fail(H2B_EINVAL, "b and x must not be NULL");
    if (overlaps(b, sizeof(double) * n, x, sizeof(double) * n)) fail(H2B_EINVAL, "b and x overlap");
    if (!(prm.tol >= 0.0) || !std::isfinite(prm.tol)) fail(H2B_EINVAL, "tol must be finite and >= 0");
    if (prm.max_iter < 0) fail(H2B_EINVAL, "max_iter must be >= 0");
    if (prm.check_every < 1) fail(H2B_EINVAL, "check_every must be >= 1");
    prepare_product(A, 1);

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
    double *r = w.r.as<double>(), *p = w.p.as<double>(), *q = w.q.as<double>();
    double *part = w.part.as<double>(), *part2 = w.part2.as<double>(), *hist = w.hist.as<double>();
    CgState *S = w.state.as<CgState>();

    // r0 = b - A x0, p0 = r0, q = 0
    if (prm.zero_guess) launch_fill_zero<double>(x, n, st);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(KT), 0, st, b, r, n);
    if (!prm.zero_guess) matvec(A, 0, -1.0, x, n, r, n, 1, st);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, b, b, n, part);
    hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, st, r, r, n, part2);
    hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(KT), 0, st, part, part2, nb, prm.tol, prm.max_iter, S, hist);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(KT), 0, st, r, p, n);
    launch_fill_zero<double>(q, n, st);
    hip_check(hipGetLastError(), "cg start");

    // the vector work of one iteration after q = A p
    auto update = [&](hipStream_t s) {
        hipLaunchKernelGGL(k_dot_part, dim3(nb), dim3(KT), 0, s, p, q, n, part);
        hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(KT), 0, s, part, nb, S);
        hipLaunchKernelGGL(k_cg_step, dim3(nb), dim3(KT), 0, s, x, r, p, q, n, S, part2);
        hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(KT), 0, s, part2, nb, S, hist);
        hipLaunchKernelGGL(k_cg_direction, dim3(nb), dim3(KT), 0, s, p, r, n, S);
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
                matvec(A, 0, 1.0, p, n, q, n, 1, w.cap);
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
                matvec(A, 0, 1.0, p, n, q, n, 1, st);
                update(st);
            }
        cur = read_state();
    }
    if (cur.status == 0) fail(H2B_EDEVICE, "conjugate gradients did not reach a stop state");
    if (history)
        hip_check(hipMemcpy(history, hist, sizeof(double) * ((size_t)cur.iter + 1), hipMemcpyDeviceToHost),
                  "history read");
    res.iterations = cur.iter;
    res.status = cur.status;
    res.rel_residual = sqrt(cur.bnorm2 > 0.0 ? cur.rho / cur.bnorm2 : cur.rho);
    res.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace h2b
