// The H-Cholesky preconditioner on the device: conversion of the H^2
// single-layer operator into an H-matrix, and the application
// z = (L L^T)^{-1} r of the factor by forward and backward substitution.
//
// Conversion.  A farfield block of the H^2 matrix is V_t S_ts V_s^T, with the
// cluster basis V_t of a parent made from its children's through the transfer
// matrices (V_t restricted to child c is V_c E_c; Section 2, eq. (transfer)),
// so the block becomes the low-rank product U V^T with U = V_t S_ts and
// V = V_s; nearfield blocks are copied.  Only the lower triangle is kept.
//
// Application.  The substitutions follow the block recursion
//   L y = r:   y_1 = L11^{-1} r_1,  r_2 -= L21 y_1,  y_2 = L22^{-1} r_2
//   L^T z = y: z_2 = L22^{-T} y_2,  y_1 -= L21^T z_2, z_1 = L11^{-T} y_1
// flattened on the host into a list of steps, each a set of independent
// tasks: a dense diagonal leaf (multiplication by the stored inverse of its
// triangular factor), the coefficients V^T y of the low-rank blocks of one
// update, or the rows of one leaf cluster that an update changes (the sum of
// its dense and low-rank parts).  The chain of diagonal leaves is sequential,
// so one workgroup runs the whole list, its 16 waves taking the tasks of a
// step and a barrier between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <chrono>
#include <unordered_map>

#include "device.hpp"
#include "hchol.hpp"
#include "linalg.hpp"

namespace h2b {

namespace {

constexpr int XW = 16;  // waves of the executor
constexpr int MAXDIAG = HProgram::MAXDIAG, TW = HProgram::TW;
constexpr int T_DIAG = HProgram::T_DIAG, T_COEF = HProgram::T_COEF, T_ROWS = HProgram::T_ROWS;
constexpr int T_SUM = HProgram::T_SUM, I_ROW = HProgram::I_ROW;

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int64_t off64(const int32_t *d) { return (int64_t)(uint32_t)d[0] | ((int64_t)d[1] << 32); }

// Runs steps [s0, s1) of the program on y (tree positions) with one
// workgroup of XW waves.
__global__ __launch_bounds__(64 * XW) void k_hchol_run(const int32_t *__restrict__ step_ptr, int s0, int s1,
                                                       const int32_t *__restrict__ tasks,
                                                       const int32_t *__restrict__ items,
                                                       const double *__restrict__ vals, double *coef, double *y)
{
    __shared__ double buf[XW][MAXDIAG];
    __shared__ double part[XW][MAXDIAG];  // per-wave partial sums of a shared task
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int s = s0; s < s1; ++s) {
        const int t0 = step_ptr[s], t1 = step_ptr[s + 1];
        // A step of one diagonal-leaf or one row task (most steps near the
        // leaves) is split over all waves: wave w sums its share of the
        // columns (diagonal leaf) or of the 16-column pieces of the items
        // (rows) for every output, and the partial sums are added in order of
        // w.  The condition is the same for every wave of the workgroup.
        const int type0 = t1 > t0 ? tasks[(int64_t)t0 * TW] : -1;
        if (t1 - t0 == 1 && (type0 == T_DIAG || type0 == T_ROWS)) {
            const int32_t *d = tasks + (int64_t)t0 * TW;
            const bool diag = d[0] == T_DIAG;
            const int o = d[1], n = d[2];
            if (diag) {
                for (int j = threadIdx.x; j < n; j += 64 * XW) buf[0][j] = y[o + j];
                __syncthreads();
                const double *M = vals + off64(d + 3);
                const int cw = (n + XW - 1) / XW, j0 = min(n, wave * cw), j1 = min(n, j0 + cw);
                for (int i = lane; i < n; i += 64) {
                    double acc = 0.0;
                    int j = j0;
                    for (; j + 4 <= j1; j += 4) {
                        double m[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) m[q] = M[(int64_t)(j + q) * n + i];
#pragma unroll
                        for (int q = 0; q < 4; ++q) acc += m[q] * buf[0][j + q];
                    }
                    for (; j < j1; ++j) acc += M[(int64_t)j * n + i] * buf[0][j];
                    part[wave][i] = acc;
                }
            } else {
                const int i0 = d[3], i1 = d[4];
                for (int e = lane; e < n; e += 64) part[wave][e] = 0.0;
                // pieces of 16 columns over all items, dealt round-robin to the waves
                int piece = 0;
                for (int it = i0; it < i1; ++it) {
                    const int32_t *m = items + (int64_t)it * TW;
                    const int nin = m[7];
                    const int np = (nin + 15) / 16;
                    const int first = (wave - piece % XW + XW) % XW;  // this wave's first piece of the item
                    if (first < np) {
                        const double *A = vals + off64(m + 1);
                        const int ld = m[3], r0 = m[4], x0 = m[6];
                        const double *src = (m[5] == 0 ? (const double *)y : (const double *)coef) + x0;
                        const int64_t st = m[0] == I_ROW ? 1 : ld;
                        for (int e = lane; e < n; e += 64) {
                            const double *a = m[0] == I_ROW ? A + (int64_t)(r0 + e) * ld : A + r0 + e;
                            double acc = 0.0;
                            for (int pc = first; pc < np; pc += XW) {
                                const int j0 = 16 * pc, j1 = min(nin, j0 + 16);
                                double av[16], sv[16];
#pragma unroll
                                for (int q = 0; q < 16; ++q) {
                                    const int j = min(j0 + q, j1 - 1);
                                    av[q] = a[(int64_t)j * st];
                                    sv[q] = j0 + q < j1 ? src[j] : 0.0;
                                }
#pragma unroll
                                for (int q = 0; q < 16; ++q) acc += av[q] * sv[q];
                            }
                            part[wave][e] += acc;
                        }
                    }
                    piece += np;
                }
            }
            __syncthreads();
            for (int i = threadIdx.x; i < n; i += 64 * XW) {
                double v = 0.0;
#pragma unroll
                for (int w = 0; w < XW; ++w) v += part[w][i];
                y[o + i] = diag ? v : y[o + i] - v;
            }
            __syncthreads();
            continue;
        }
        for (int ti = t0 + wave; ti < t1; ti += XW) {
            const int32_t *d = tasks + (int64_t)ti * TW;
            const int type = d[0];
            if (type == T_DIAG) {
                // y[o .. o+n) = M^T-indexed product: out_i = sum_j M[j n + i] y_j
                const int o = d[1], n = d[2];
                const double *M = vals + off64(d + 3);
                for (int j = lane; j < n; j += 64) buf[wave][j] = y[o + j];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (int i = lane; i < n; i += 64) {
                    // 8 independent loads per batch, summed in order of j
                    double acc = 0.0;
                    int j = 0;
                    for (; j + 8 <= n; j += 8) {
                        double m[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) m[q] = M[(int64_t)(j + q) * n + i];
#pragma unroll
                        for (int q = 0; q < 8; ++q) acc += m[q] * buf[wave][j + q];
                    }
                    for (; j < n; ++j) acc += M[(int64_t)j * n + i] * buf[wave][j];
                    y[o + i] = acc;
                }
                // the next task of this wave may overwrite buf
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            } else if (type == T_SUM) {
                // coef[dst + p] = sum over the pieces of their partial coefficients, in order
                const int dst = d[1], src = d[2], np = d[3], k = d[5];
                for (int p = lane; p < k; p += 64) {
                    double acc = 0.0;
                    for (int q = 0; q < np; ++q) acc += coef[src + (int64_t)q * k + p];
                    coef[dst + p] = acc;
                }
            } else if (type == T_COEF) {
                // coef[c .. c+k) = M^T y[yo .. yo+len), M (len x k)
                const int yo = d[1], len = d[2];
                const double *M = vals + off64(d + 3);
                const int k = d[5], c = d[6];
                for (int p0 = 0; p0 < k; p0 += 8) {
                    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                    for (int j = lane; j < len; j += 64) {
                        // all 9 loads issued together (columns past k clamped, weight 0)
                        const double yj = y[yo + j];
                        const double *m = M + (int64_t)j * k;
                        double mv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) mv[q] = m[min(p0 + q, k - 1)];
#pragma unroll
                        for (int q = 0; q < 8; ++q) acc[q] += (p0 + q < k ? mv[q] : 0.0) * yj;
                    }
#pragma unroll
                    for (int q = 0; q < 8; ++q) acc[q] = wave_sum(acc[q]);
                    if (lane < 8 && p0 + lane < k) {
                        double v = acc[0];
#pragma unroll
                        for (int q = 1; q < 8; ++q)
                            if (lane == q) v = acc[q];
                        coef[c + p0 + lane] = v;
                    }
                }
            } else {
                // y[o + e] -= sum over items of sum_j M(e, j) src[x0 + j]
                const int o = d[1], len = d[2], i0 = d[3], i1 = d[4];
                for (int e0 = 0; e0 < len; e0 += 64) {
                    const int e = e0 + lane;
                    double acc = 0.0;
                    if (e < len) {
                        for (int it = i0; it < i1; ++it) {
                            const int32_t *m = items + (int64_t)it * TW;
                            const double *A = vals + off64(m + 1);
                            const int ld = m[3], r0 = m[4], x0 = m[6], nin = m[7];
                            const double *src = (m[5] == 0 ? (const double *)y : (const double *)coef) + x0;
                            // stride between consecutive j: 1 (rows) or ld (columns);
                            // 8 independent pairs of loads per batch, summed in order
                            const double *a = m[0] == I_ROW ? A + (int64_t)(r0 + e) * ld : A + r0 + e;
                            const int64_t st = m[0] == I_ROW ? 1 : ld;
                            int j = 0;
                            for (; j + 8 <= nin; j += 8) {
                                double av[8], sv[8];
#pragma unroll
                                for (int q = 0; q < 8; ++q) {
                                    av[q] = a[(int64_t)(j + q) * st];
                                    sv[q] = src[j + q];
                                }
#pragma unroll
                                for (int q = 0; q < 8; ++q) acc += av[q] * sv[q];
                            }
                            for (; j < nin; ++j) acc += a[(int64_t)j * st] * src[j];
                        }
                        y[o + e] -= acc;
                    }
                }
            }
        }
        __syncthreads();
    }
}

__global__ void k_hchol_gather(const int32_t *__restrict__ perm, int64_t n, const double *__restrict__ r,
                               double *__restrict__ y)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = r[perm[i]];
}

__global__ void k_hchol_scatter(const int32_t *__restrict__ perm, int64_t n, const double *__restrict__ y,
                                double *__restrict__ z)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[perm[i]] = y[i];
}

inline int grid_of(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 4096); }

}  // namespace

std::unique_ptr<HMatrix> hmatrix_from_op(const Op &op, double eps, hipStream_t st)
{
    if (op.kernel != H2B_SLP) fail(H2B_EINVAL, "the H-Cholesky preconditioner is built for the single-layer operator");
    if (op.rowb != op.colb || op.blocks->rows != op.blocks->cols)
        fail(H2B_ENOTSUP, "the H-Cholesky preconditioner needs the operator on one cluster tree");
    if (op.params.farfield_dtype != H2B_F64) fail(H2B_ENOTSUP, "the H-Cholesky preconditioner needs the FP64 far field");
    if (op.recompute) fail(H2B_ENOTSUP, "the H-Cholesky preconditioner needs stored coupling matrices");
    const Basis &B = *op.rowb;
    const Tree &T = *B.tree;
    const int64_t nc = T.nclusters();
    auto download = [&](const DevMem &m, int64_t count) {
        std::vector<double> h((size_t)std::max<int64_t>(count, 0));
        if (count > 0)
            hip_check(hipMemcpyAsync(h.data(), m.p, sizeof(double) * count, hipMemcpyDeviceToHost, st), "download");
        return h;
    };
    const std::vector<double> leafv = download(B.leaf_vals, B.leaf.total);
    const std::vector<double> transv = download(B.trans_vals, B.trans.total);
    const std::vector<double> cplv = download(op.cpl_vals, op.cpl.total);
    const std::vector<double> nearv = download(op.near_vals, op.near.total);
    hip_check(hipStreamSynchronize(st), "download");

    // explicit cluster bases V_c (|c| x k_c), leaves first, then parents up
    std::vector<std::vector<double>> V(nc);
    for (int g = 0; g < B.leaf.ngroups(); ++g) {
        const int c = B.leaf.group_tag[g], k = B.rank[c], n = T.size(c);
        const int q = B.leaf.seg_ptr[g];
        if (B.leaf.seg_in[q] != T.begin[c] || B.leaf.seg_len[q] != n) fail(H2B_EDEVICE, "unexpected leaf panel");
        const double *P = &leafv[B.leaf.val_off[g]];  // k x n = V^T
        V[c].assign((size_t)n * k, 0.0);
        for (int p = 0; p < k; ++p)
            for (int i = 0; i < n; ++i) V[c][(size_t)i * k + p] = P[(size_t)p * n + i];
    }
    for (int g = 0; g < B.trans.ngroups(); ++g) {  // deepest parents first
        const int t = B.trans.group_tag[g], kt = B.rank[t], n = T.size(t), nc_g = B.trans.ncols[g];
        const double *P = &transv[B.trans.val_off[g]];  // kt x (k_c0 + k_c1) = [E_c0^T | E_c1^T]
        V[t].assign((size_t)n * kt, 0.0);
        for (int q = B.trans.seg_ptr[g]; q < B.trans.seg_ptr[g + 1]; ++q) {
            const int c = B.trans.seg_tag[q], kc = B.rank[c], c0 = B.trans.seg_c0[q];
            if (kc == 0) continue;
            if ((int64_t)V[c].size() != (int64_t)T.size(c) * kc) fail(H2B_EDEVICE, "child basis missing");
            const int ro = T.begin[c] - T.begin[t];
            for (int i = 0; i < T.size(c); ++i)
                for (int p = 0; p < kt; ++p) {
                    double s = 0.0;
                    for (int r = 0; r < kc; ++r) s += V[c][(size_t)i * kc + r] * P[(size_t)p * nc_g + c0 + r];
                    V[t][(size_t)(ro + i) * kt + p] = s;
                }
        }
    }

    std::vector<int> fn, nn;
    auto H = hmatrix_structure(*op.blocks, fn, nn);
    H->eps = eps;
    std::unordered_map<int64_t, int> node_of;
    for (size_t b = 0; b < fn.size(); ++b)
        if (fn[b] >= 0) node_of[(int64_t)op.blocks->far_t[b] * nc + op.blocks->far_s[b]] = fn[b];
    for (size_t b = 0; b < nn.size(); ++b)
        if (nn[b] >= 0) node_of[(int64_t)op.blocks->near_t[b] * nc + op.blocks->near_s[b]] = nn[b];
    // far blocks: U = V_t S_ts, V = V_s
    for (int g = 0; g < op.cpl.ngroups(); ++g) {
        const int t = op.cpl.group_tag[g], kt = B.rank[t], ncol = op.cpl.ncols[g];
        const double *P = &cplv[op.cpl.val_off[g]];
        for (int q = op.cpl.seg_ptr[g]; q < op.cpl.seg_ptr[g + 1]; ++q) {
            const int s = op.cpl.seg_tag[q], ks = B.rank[s], c0 = op.cpl.seg_c0[q];
            auto it = node_of.find((int64_t)t * nc + s);
            if (it == node_of.end()) continue;  // upper triangle
            HNode &N = H->nodes[it->second];
            const int nt = T.size(t), ns = T.size(s);
            N.k = ks;
            N.a.assign((size_t)nt * ks, 0.0);
            for (int i = 0; i < nt; ++i)
                for (int p = 0; p < kt; ++p) {
                    const double v = V[t][(size_t)i * kt + p];
                    if (v == 0.0) continue;
                    for (int r = 0; r < ks; ++r) N.a[(size_t)i * ks + r] += v * P[(size_t)p * ncol + c0 + r];
                }
            N.b = V[s];
            if ((int64_t)N.b.size() != (int64_t)ns * ks) fail(H2B_EDEVICE, "column basis missing");
        }
    }
    // near blocks
    for (int g = 0; g < op.near.ngroups(); ++g) {
        const int t = op.near.group_tag[g], nt = op.near.nrows[g], ncol = op.near.ncols[g];
        const double *P = &nearv[op.near.val_off[g]];
        for (int q = op.near.seg_ptr[g]; q < op.near.seg_ptr[g + 1]; ++q) {
            const int s = op.near.seg_tag[q], ns = op.near.seg_len[q], c0 = op.near.seg_c0[q];
            auto it = node_of.find((int64_t)t * nc + s);
            if (it == node_of.end()) continue;
            HNode &N = H->nodes[it->second];
            for (int i = 0; i < nt; ++i)
                for (int j = 0; j < ns; ++j) N.a[(size_t)i * ns + j] = P[(size_t)i * ncol + c0 + j];
        }
    }
    return H;
}

void hchol_factor(HChol &P, double eps)
{
    const auto t0 = std::chrono::steady_clock::now();
    hmatrix_coarsen(*P.H, eps);
    const auto t1 = std::chrono::steady_clock::now();
    P.coarse = hmatrix_stats(*P.H);
    hmatrix_cholesky(*P.H);
    const auto t2 = std::chrono::steady_clock::now();
    P.factor = hmatrix_stats(*P.H);
    P.coarsen_s = std::chrono::duration<double>(t1 - t0).count();
    P.factor_s = std::chrono::duration<double>(t2 - t1).count();
}

void hchol_flatten(HChol &P)
{
    if (P.prog_host.built) return;
    hprogram_build(*P.H, P.prog_host);
}

void hchol_upload(HChol &P, hipStream_t st)
{
    if (P.uploaded) return;
    hchol_flatten(P);
    HProgram &F = P.prog_host;
    const Tree &T = *P.H->tree;
    P.n = T.n;
    P.nsteps = (int)F.step_ptr.size() - 1;
    P.fw_steps = F.fw_steps;
    P.ntasks = (int64_t)F.tasks.size() / TW;
    P.vals.alloc(sizeof(double) * std::max<size_t>(F.vals.size(), 1));
    hip_check(hipMemcpyAsync(P.vals.p, F.vals.data(), sizeof(double) * F.vals.size(), hipMemcpyHostToDevice, st),
              "upload");
    P.coef.alloc(sizeof(double) * std::max<int64_t>(F.ncoef, 1));
    P.y.alloc(sizeof(double) * std::max<int64_t>(P.n, 1));
    Packer pk;
    std::vector<int32_t> pad(TW, 0);
    pk.add(F.step_ptr, const_cast<int32_t **>(&P.d_step));
    pk.add(F.tasks.empty() ? pad : F.tasks, const_cast<int32_t **>(&P.d_tasks));
    pk.add(F.items.empty() ? pad : F.items, const_cast<int32_t **>(&P.d_items));
    pk.add(T.perm, const_cast<int32_t **>(&P.d_perm));
    pk.upload(P.prog, st);
    hip_check(hipStreamSynchronize(st), "upload");
    P.device_values = (int64_t)F.vals.size();
    P.uploaded = true;
}

void hchol_apply(HChol &P, const double *r, double *z, hipStream_t st)
{
    if (!P.uploaded) fail(H2B_ESTATE, "the preconditioner is not on the device");
    double *y = P.y.as<double>();
    hipLaunchKernelGGL(k_hchol_gather, dim3(grid_of(P.n)), dim3(256), 0, st, P.d_perm, P.n, r, y);
    if (P.nsteps > 0)
        hipLaunchKernelGGL(k_hchol_run, dim3(1), dim3(64 * XW), 0, st, P.d_step, 0, P.nsteps, P.d_tasks, P.d_items,
                           P.vals.as<double>(), P.coef.as<double>(), y);
    hipLaunchKernelGGL(k_hchol_scatter, dim3(grid_of(P.n)), dim3(256), 0, st, P.d_perm, P.n, y, z);
    hip_check(hipGetLastError(), "preconditioner launch");
}

}  // namespace h2b
