// Algebraic recompression of the interpolation H^2 matrix: orthogonalise the
// nested cluster bases, weight every cluster by all farfield blocks that use
// it (its own and its ancestors'), truncate each cluster's weighted basis to a
// relative tolerance, and project the coupling matrices onto the new bases.
//
// The paper turns its cross-approximation matrices into H^2 form with the
// algebraic compression of its reference [BO07a] (Section 3; Section 5 notes it
// yields close to the best H^2 approximation); here the same idea is applied
// to an H^2 matrix with nested bases, from interpolation or from the Green
// cross approximation (any per-cluster ranks):
//   1. V_t = Q_t R_t with Q_t orthonormal and nested (QR bottom-up, from the
//      stored leaf and transfer matrices);
//   2. S~_ts = R_t S_ts R'_s^T (GPU);
//   3. Gram weights Z_t = sum_s S~_ts S~_ts^T + F_t Z_parent F_t^T (GPU sums,
//      host recursion top-down);
//   4. bottom-up: eigenvectors of the weighted (projected) basis, keep the
//      directions with sigma_i > tol * sigma_1 of that cluster;
//   5. S''_ts = B_t S~_ts B'_s^T with B_t = Q''_t^T Q_t (GPU).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "linalg.hpp"
#include "op.hpp"

namespace h2b {

namespace {

constexpr int RK = 64;  // tile of the recompression kernels (larger blocks: the tiled kernels)
constexpr int NT = 256;

struct SandwichDev {
    const int64_t *in_off, *out_off;
    const int32_t *in_stride, *out_stride, *a_in, *b_in, *a_out, *b_out, *t, *s;
};

// out = L_t * In * R_s^T for one block per workgroup.
template <typename TO>
__global__ __launch_bounds__(NT) void k_sandwich(SandwichDev d, const double *__restrict__ in,
                                                 TO *__restrict__ out, const double *__restrict__ L,
                                                 const int64_t *__restrict__ Loff,
                                                 const double *__restrict__ R,
                                                 const int64_t *__restrict__ Roff)
{
    __shared__ double X[RK * RK];
    __shared__ double T[RK * RK];
    const int b = blockIdx.x;
    const int ai = d.a_in[b], bi = d.b_in[b], ao = d.a_out[b], bo = d.b_out[b];
    const int64_t io = d.in_off[b], oo = d.out_off[b];
    const int is = d.in_stride[b], os = d.out_stride[b];
    for (int e = threadIdx.x; e < ai * bi; e += NT) X[e] = in[io + (int64_t)(e / bi) * is + e % bi];
    __syncthreads();
    const double *Lt = L + Loff[d.t[b]];
    for (int e = threadIdx.x; e < ao * bi; e += NT) {
        const int i = e / bi, c = e % bi;
        double s = 0.0;
        for (int j = 0; j < ai; ++j) s += Lt[i * ai + j] * X[j * bi + c];
        T[e] = s;
    }
    __syncthreads();
    const double *Rs = R + Roff[d.s[b]];
    for (int e = threadIdx.x; e < ao * bo; e += NT) {
        const int i = e / bo, c = e % bo;
        double s = 0.0;
        for (int j = 0; j < bi; ++j) s += T[i * bi + j] * Rs[c * bi + j];
        out[oo + (int64_t)i * os + c] = (TO)s;
    }
}

// Gram of each row panel: Z = P P^T (nrows x nrows).
__global__ __launch_bounds__(NT) void k_gram_rows(RowPanelDev d, const double *__restrict__ vals,
                                                  double *__restrict__ gram,
                                                  const int64_t *__restrict__ goff)
{
    __shared__ double C[RK][RK + 1];
    const int g = blockIdx.x;
    const int a = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    double acc[RK * RK / NT];
    for (int k = 0; k < RK * RK / NT; ++k) acc[k] = 0.0;
    for (int c0 = 0; c0 < nc; c0 += RK) {
        const int cl = min(RK, nc - c0);
        for (int e = threadIdx.x; e < RK * RK; e += NT) {
            const int i = e / RK, j = e % RK;
            C[i][j] = (i < a && j < cl) ? vals[off + (int64_t)i * nc + c0 + j] : 0.0;
        }
        __syncthreads();
        for (int k = 0; k < RK * RK / NT; ++k) {
            const int e = threadIdx.x + k * NT;
            const int i = e / RK, j = e % RK;
            double s = 0.0;
            for (int jj = 0; jj < RK; ++jj) s += C[i][jj] * C[j][jj];
            acc[k] += s;
        }
        __syncthreads();
    }
    double *G = gram + goff[d.tag[g]];
    for (int k = 0; k < RK * RK / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int i = e / RK, j = e % RK;
        if (i < a && j < a) G[i * a + j] = acc[k];
    }
}

// Gram of each column group: Z = sum over blocks of B^T B (out_len x out_len).
__global__ __launch_bounds__(NT) void k_gram_cols(ColPanelDev d, const double *__restrict__ vals,
                                                  double *__restrict__ gram,
                                                  const int64_t *__restrict__ goff,
                                                  const int32_t *__restrict__ gtag)
{
    __shared__ double C[RK][RK + 1];
    const int g = blockIdx.x;
    const int b = d.out_len[g];
    double acc[RK * RK / NT];
    for (int k = 0; k < RK * RK / NT; ++k) acc[k] = 0.0;
    for (int blk = d.blk_ptr[g]; blk < d.blk_ptr[g + 1]; ++blk) {
        const int nr = d.b_nrows[blk];
        const int64_t stride = d.b_stride[blk];
        const double *base = vals + d.b_val_off[blk] + d.b_c0[blk];
        for (int r0 = 0; r0 < nr; r0 += RK) {
            const int rl = min(RK, nr - r0);
            for (int e = threadIdx.x; e < RK * RK; e += NT) {
                const int r = e / RK, j = e % RK;
                C[r][j] = (r < rl && j < b) ? base[(int64_t)(r0 + r) * stride + j] : 0.0;
            }
            __syncthreads();
            for (int k = 0; k < RK * RK / NT; ++k) {
                const int e = threadIdx.x + k * NT;
                const int i = e / RK, j = e % RK;
                double s = 0.0;
                for (int r = 0; r < RK; ++r) s += C[r][i] * C[r][j];
                acc[k] += s;
            }
            __syncthreads();
        }
    }
    double *G = gram + goff[gtag[g]];
    for (int k = 0; k < RK * RK / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int i = e / RK, j = e % RK;
        if (i < b && j < b) G[i * b + j] = acc[k];
    }
}

// ------------------------------------------------ ranks above RK
//
// The same three products for blocks with a dimension above RK (orders 5-6,
// cross-approximation bases): tiles of RK x RK held in LDS, accumulators in
// registers per tile, one workgroup per (block, output tile).

constexpr int GT = 32;  // rows (sandwich) or columns (Gram) staged per step

// out = L * In * R^T, FP64 output, for one output tile of RK x RK of one block
// per workgroup: U = In[j0:j0+GT, :] R^T[:, tile] is staged in LDS for GT rows
// of In at a time, then out[tile] += L[tile, j0:j0+GT] U.
__global__ __launch_bounds__(NT) void k_sandwich_tiled(SandwichDev d, int tiles, const double *__restrict__ in,
                                                       double *__restrict__ out, const double *__restrict__ L,
                                                       const int64_t *__restrict__ Loff,
                                                       const double *__restrict__ R,
                                                       const int64_t *__restrict__ Roff)
{
    __shared__ double U[GT][RK + 1];
    __shared__ double Lc[RK][GT + 1];
    const int b = blockIdx.x / (tiles * tiles), tile = blockIdx.x % (tiles * tiles);
    const int ai = d.a_in[b], bi = d.b_in[b], ao = d.a_out[b], bo = d.b_out[b];
    const int i0 = (tile / tiles) * RK, c0 = (tile % tiles) * RK;
    if (i0 >= ao || c0 >= bo) return;  // uniform over the workgroup
    const int64_t io = d.in_off[b], oo = d.out_off[b];
    const int is = d.in_stride[b], os = d.out_stride[b];
    const double *Lt = L + Loff[d.t[b]];
    const double *Rs = R + Roff[d.s[b]];
    double acc[RK * RK / NT];
    for (int k = 0; k < RK * RK / NT; ++k) acc[k] = 0.0;
    for (int j0 = 0; j0 < ai; j0 += GT) {
        // U[jj][c] = sum_l In[j0 + jj][l] R[c0 + c][l]
        for (int e = threadIdx.x; e < GT * RK; e += NT) {
            const int jj = e / RK, c = e % RK;
            double sum = 0.0;
            if (j0 + jj < ai && c0 + c < bo) {
                const double *x = in + io + (int64_t)(j0 + jj) * is;
                const double *r = Rs + (int64_t)(c0 + c) * bi;
                for (int l = 0; l < bi; ++l) sum += x[l] * r[l];
            }
            U[jj][c] = sum;
        }
        for (int e = threadIdx.x; e < RK * GT; e += NT) {
            const int i = e / GT, jj = e % GT;
            Lc[i][jj] = (i0 + i < ao && j0 + jj < ai) ? Lt[(int64_t)(i0 + i) * ai + j0 + jj] : 0.0;
        }
        __syncthreads();
        for (int k = 0; k < RK * RK / NT; ++k) {
            const int e = threadIdx.x + k * NT;
            const int i = e / RK, c = e % RK;
            double sum = 0.0;
            for (int jj = 0; jj < GT; ++jj) sum += Lc[i][jj] * U[jj][c];
            acc[k] += sum;
        }
        __syncthreads();
    }
    for (int k = 0; k < RK * RK / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int i = e / RK, c = e % RK;
        if (i0 + i < ao && c0 + c < bo) out[oo + (int64_t)(i0 + i) * os + c0 + c] = acc[k];
    }
}

// Gram of each row panel, Z = P P^T, one RK x RK tile (i0, j0) per workgroup.
__global__ __launch_bounds__(NT) void k_gram_rows_tiled(RowPanelDev d, int tiles, const double *__restrict__ vals,
                                                        double *__restrict__ gram,
                                                        const int64_t *__restrict__ goff)
{
    __shared__ double Ci[RK][GT + 1], Cj[RK][GT + 1];
    const int g = blockIdx.x / (tiles * tiles), tile = blockIdx.x % (tiles * tiles);
    const int a = d.nrows[g], nc = d.ncols[g];
    const int i0 = (tile / tiles) * RK, j0 = (tile % tiles) * RK;
    if (i0 >= a || j0 >= a) return;  // uniform over the workgroup
    const int64_t off = d.val_off[g];
    double acc[RK * RK / NT];
    for (int k = 0; k < RK * RK / NT; ++k) acc[k] = 0.0;
    for (int c0 = 0; c0 < nc; c0 += GT) {
        for (int e = threadIdx.x; e < RK * GT; e += NT) {
            const int r = e / GT, c = e % GT;
            const bool in = c0 + c < nc;
            Ci[r][c] = (in && i0 + r < a) ? vals[off + (int64_t)(i0 + r) * nc + c0 + c] : 0.0;
            Cj[r][c] = (in && j0 + r < a) ? vals[off + (int64_t)(j0 + r) * nc + c0 + c] : 0.0;
        }
        __syncthreads();
        for (int k = 0; k < RK * RK / NT; ++k) {
            const int e = threadIdx.x + k * NT;
            const int i = e / RK, j = e % RK;
            double sum = 0.0;
            for (int c = 0; c < GT; ++c) sum += Ci[i][c] * Cj[j][c];
            acc[k] += sum;
        }
        __syncthreads();
    }
    double *G = gram + goff[d.tag[g]];
    for (int k = 0; k < RK * RK / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int i = e / RK, j = e % RK;
        if (i0 + i < a && j0 + j < a) G[(int64_t)(i0 + i) * a + j0 + j] = acc[k];
    }
}

// Gram of each column group, Z = sum over blocks of B^T B, one RK x RK tile
// (i0, j0) per workgroup.
__global__ __launch_bounds__(NT) void k_gram_cols_tiled(ColPanelDev d, int tiles, const double *__restrict__ vals,
                                                        double *__restrict__ gram,
                                                        const int64_t *__restrict__ goff,
                                                        const int32_t *__restrict__ gtag)
{
    __shared__ double Ci[GT][RK + 1], Cj[GT][RK + 1];
    const int g = blockIdx.x / (tiles * tiles), tile = blockIdx.x % (tiles * tiles);
    const int b = d.out_len[g];
    const int i0 = (tile / tiles) * RK, j0 = (tile % tiles) * RK;
    if (i0 >= b || j0 >= b) return;  // uniform over the workgroup
    double acc[RK * RK / NT];
    for (int k = 0; k < RK * RK / NT; ++k) acc[k] = 0.0;
    for (int blk = d.blk_ptr[g]; blk < d.blk_ptr[g + 1]; ++blk) {
        const int nr = d.b_nrows[blk];
        const int64_t stride = d.b_stride[blk];
        const double *base = vals + d.b_val_off[blk] + d.b_c0[blk];
        for (int r0 = 0; r0 < nr; r0 += GT) {
            for (int e = threadIdx.x; e < GT * RK; e += NT) {
                const int r = e / RK, j = e % RK;
                const bool in = r0 + r < nr;
                Ci[r][j] = (in && i0 + j < b) ? base[(int64_t)(r0 + r) * stride + i0 + j] : 0.0;
                Cj[r][j] = (in && j0 + j < b) ? base[(int64_t)(r0 + r) * stride + j0 + j] : 0.0;
            }
            __syncthreads();
            for (int k = 0; k < RK * RK / NT; ++k) {
                const int e = threadIdx.x + k * NT;
                const int i = e / RK, j = e % RK;
                double sum = 0.0;
                for (int r = 0; r < GT; ++r) sum += Ci[r][i] * Cj[r][j];
                acc[k] += sum;
            }
            __syncthreads();
        }
    }
    double *G = gram + goff[gtag[g]];
    for (int k = 0; k < RK * RK / NT; ++k) {
        const int e = threadIdx.x + k * NT;
        const int i = e / RK, j = e % RK;
        if (i0 + i < b && j0 + j < b) G[(int64_t)(i0 + i) * b + j0 + j] = acc[k];
    }
}

// ----------------------------------------------------------------- host

// Orthogonalised cluster basis: V_t = Q_t R_t, Q_parent|_c = Q_c F_c.
struct Ortho {
    std::vector<int> r;                     // rank after orthogonalisation
    std::vector<std::vector<double>> R;     // r_t x k
    std::vector<std::vector<double>> Q;     // leaves: |t| x r_t
    std::vector<std::vector<double>> F;     // non-root: r_c x r_parent
    std::vector<std::vector<double>> Z;     // weight Gram, r_t x r_t
    // truncation
    std::vector<int> kk;                    // new rank
    std::vector<std::vector<double>> B;     // k'_t x r_t  (new basis^T * old basis)
    std::vector<std::vector<double>> newleaf;  // leaves: k'_t x |t|  (new basis, transposed)
    std::vector<std::vector<double>> newtr;    // parents: k'_t x (k'_c0 + k'_c1)
};

// V_t = Q_t R_t bottom-up from the stored basis values: a leaf's V_t is its
// stored panel transposed (|t| x k_t); a parent's is [V_c0 E_c0; V_c1 E_c1]
// with E_c (k_c x k_t) read from its stored transfer panel [E_c0^T | E_c1^T],
// so Q_t restricted to child c is Q_c F_c with [F_c0; F_c1] R_t the QR of
// [R_c0 E_c0; R_c1 E_c1].  Works for any per-cluster ranks (interpolation
// k = m^3, or the cross approximation's).
void orthogonalise(const Basis &B, const std::vector<double> &leafT, const std::vector<double> &trT, Ortho &o)
{
    const Tree &T = *B.tree;
    const int64_t nc = T.nclusters();
    o.r.assign(nc, 0);
    o.R.assign(nc, {});
    o.Q.assign(nc, {});
    o.F.assign(nc, {});
    std::vector<int> leaf_g(nc, -1), tr_g(nc, -1);
    for (int g = 0; g < B.leaf.ngroups(); ++g) leaf_g[B.leaf.group_tag[g]] = g;
    for (int g = 0; g < B.trans.ngroups(); ++g) tr_g[B.trans.group_tag[g]] = g;
    for (int lev = T.nlevels - 1; lev >= 0; --lev) {
        const auto &cl = T.by_level[lev];
        parallel_for((int64_t)cl.size(), [&](int64_t idx) {
            const int c = cl[idx];
            const int kc = B.rank[c];
            if (T.nchild[c] == 0) {
                const int n = T.size(c);
                const int g = leaf_g[c];
                if (kc == 0 || n == 0 || g < 0) return;  // rank 0
                if (B.leaf.nrows[g] != kc || B.leaf.ncols[g] != n) fail(H2B_EDEVICE, "leaf panel of unexpected shape");
                std::vector<double> V((size_t)n * kc);
                const double *src = &leafT[B.leaf.val_off[g]];  // kc x n
                for (int nu = 0; nu < kc; ++nu)
                    for (int i = 0; i < n; ++i) V[(size_t)i * kc + nu] = src[(size_t)nu * n + i];
                householder_qr(n, kc, V.data(), o.Q[c], o.R[c]);
                o.r[c] = std::min(n, kc);
                return;
            }
            const int ch[2] = {T.child0[c], T.child1[c]};
            const int r0 = o.r[ch[0]], r1 = o.r[ch[1]];
            const int g = tr_g[c];
            if (kc == 0 || r0 + r1 == 0 || g < 0) {  // rank 0: the children's F have no columns
                o.F[ch[0]].clear();
                o.F[ch[1]].clear();
                return;
            }
            if (B.trans.nrows[g] != kc) fail(H2B_EDEVICE, "transfer panel of unexpected shape");
            const int ncol = B.trans.ncols[g];
            const double *P = &trT[B.trans.val_off[g]];  // kc x ncol
            std::vector<double> W((size_t)(r0 + r1) * kc, 0.0);
            int roff = 0;
            for (int q = 0; q < 2; ++q) {
                const int cc = ch[q], rq = o.r[cc], kq = B.rank[cc];
                if (rq > 0) {
                    int seg = -1;
                    for (int j = B.trans.seg_ptr[g]; j < B.trans.seg_ptr[g + 1]; ++j)
                        if (B.trans.seg_tag[j] == cc) seg = j;
                    if (seg < 0 || B.trans.seg_len[seg] != kq) fail(H2B_EDEVICE, "transfer segment of unexpected shape");
                    const int s0 = B.trans.seg_c0[seg];
                    std::vector<double> E((size_t)kq * kc);  // E[mu][nu] = P[nu][s0 + mu]
                    for (int mu = 0; mu < kq; ++mu)
                        for (int nu = 0; nu < kc; ++nu) E[(size_t)mu * kc + nu] = P[(size_t)nu * ncol + s0 + mu];
                    gemm_nn(rq, kc, kq, o.R[cc].data(), E.data(), W.data() + (size_t)roff * kc);
                }
                roff += rq;
            }
            std::vector<double> Qh;
            householder_qr(r0 + r1, kc, W.data(), Qh, o.R[c]);
            const int rc = std::min(r0 + r1, kc);
            o.r[c] = rc;
            o.F[ch[0]].assign(Qh.begin(), Qh.begin() + (size_t)r0 * rc);
            o.F[ch[1]].assign(Qh.begin() + (size_t)r0 * rc, Qh.end());
        });
    }
}

// Adds the ancestors' weights: Z_c += F_c Z_parent F_c^T, top-down.
void propagate_weights(const Tree &T, Ortho &o)
{
    for (int lev = 1; lev < T.nlevels; ++lev) {
        const auto &cl = T.by_level[lev];
        parallel_for((int64_t)cl.size(), [&](int64_t idx) {
            const int c = cl[idx];
            const int p = T.parent[c];
            const int rc = o.r[c], rp = o.r[p];
            std::vector<double> tmp((size_t)rc * rp), add((size_t)rc * rc);
            gemm_nn(rc, rp, rp, o.F[c].data(), o.Z[p].data(), tmp.data());
            gemm_nt(rc, rc, rp, tmp.data(), o.F[c].data(), add.data());
            for (size_t i = 0; i < add.size(); ++i) o.Z[c][i] += add[i];
        });
    }
}

// Eigen-decomposition of the symmetric n x n matrix M; returns the number of
// eigenvalues above tol^2 times the largest, and the leading eigenvectors as
// columns of U (n x kept).
int truncate_sym(int n, std::vector<double> M, double tol, std::vector<double> &U)
{
    if (n == 0) {
        U.clear();
        return 0;
    }
    // symmetrise against rounding
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double v = 0.5 * (M[(size_t)i * n + j] + M[(size_t)j * n + i]);
            M[(size_t)i * n + j] = M[(size_t)j * n + i] = v;
        }
    std::vector<double> ev, Z;
    sym_eig(n, M, ev, Z);
    int kept = 0;
    if (ev[0] > 0.0) {
        const double thr = tol * tol * ev[0];
        while (kept < n && ev[kept] > thr) ++kept;
    }
    U.assign((size_t)n * kept, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < kept; ++j) U[(size_t)i * kept + j] = Z[(size_t)i * n + j];
    return kept;
}

void truncate_basis(const Tree &T, double tol, Ortho &o)
{
    const int64_t nc = T.nclusters();
    o.kk.assign(nc, 0);
    o.B.assign(nc, {});
    o.newleaf.assign(nc, {});
    o.newtr.assign(nc, {});
    for (int lev = T.nlevels - 1; lev >= 0; --lev) {
        const auto &cl = T.by_level[lev];
        parallel_for((int64_t)cl.size(), [&](int64_t idx) {
            const int c = cl[idx];
            const int rc = o.r[c];
            if (T.nchild[c] == 0) {
                std::vector<double> U;
                const int kk = truncate_sym(rc, o.Z[c], tol, U);
                o.kk[c] = kk;
                // B = U^T (kk x rc)
                o.B[c].assign((size_t)kk * rc, 0.0);
                for (int i = 0; i < kk; ++i)
                    for (int j = 0; j < rc; ++j) o.B[c][(size_t)i * rc + j] = U[(size_t)j * kk + i];
                // new leaf basis Q U (n x kk), stored transposed (kk x n)
                const int n = T.size(c);
                std::vector<double> QU((size_t)n * kk);
                gemm_nn(n, kk, rc, o.Q[c].data(), U.data(), QU.data());
                o.newleaf[c].assign((size_t)kk * n, 0.0);
                for (int i = 0; i < n; ++i)
                    for (int j = 0; j < kk; ++j) o.newleaf[c][(size_t)j * n + i] = QU[(size_t)i * kk + j];
            } else {
                const int c0 = T.child0[c], c1 = T.child1[c];
                const int k0 = o.kk[c0], k1 = o.kk[c1];
                const int nrow = k0 + k1;
                // That = [B_c0 F_c0; B_c1 F_c1]  (nrow x rc)
                std::vector<double> Th((size_t)nrow * rc);
                gemm_nn(k0, rc, o.r[c0], o.B[c0].data(), o.F[c0].data(), Th.data());
                gemm_nn(k1, rc, o.r[c1], o.B[c1].data(), o.F[c1].data(), Th.data() + (size_t)k0 * rc);
                std::vector<double> tmp((size_t)nrow * rc), M((size_t)nrow * nrow);
                gemm_nn(nrow, rc, rc, Th.data(), o.Z[c].data(), tmp.data());
                gemm_nt(nrow, nrow, rc, tmp.data(), Th.data(), M.data());
                std::vector<double> U;
                const int kk = truncate_sym(nrow, M, tol, U);
                o.kk[c] = kk;
                // B = U^T That (kk x rc)
                o.B[c].assign((size_t)kk * rc, 0.0);
                gemm_tn(kk, rc, nrow, U.data(), Th.data(), o.B[c].data());
                // transfer panel = U^T (kk x nrow)
                o.newtr[c].assign((size_t)kk * nrow, 0.0);
                for (int i = 0; i < nrow; ++i)
                    for (int j = 0; j < kk; ++j) o.newtr[c][(size_t)j * nrow + i] = U[(size_t)i * kk + j];
            }
        });
    }
}

// Concatenates per-cluster matrices into one device array with offsets.
void upload_blocks(const std::vector<std::vector<double>> &mats, DevMem &vals, DevMem &offs,
                   hipStream_t st)
{
    std::vector<int64_t> off(mats.size());
    int64_t tot = 0;
    for (size_t c = 0; c < mats.size(); ++c) {
        off[c] = tot;
        tot += (int64_t)mats[c].size();
    }
    std::vector<double> flat((size_t)std::max<int64_t>(tot, 1));
    for (size_t c = 0; c < mats.size(); ++c)
        std::copy(mats[c].begin(), mats[c].end(), flat.begin() + off[c]);
    vals.alloc(flat.size() * sizeof(double));
    offs.alloc(off.size() * sizeof(int64_t) + 8);
    hip_check(hipMemcpyAsync(vals.p, flat.data(), flat.size() * sizeof(double), hipMemcpyHostToDevice, st),
              "upload");
    hip_check(hipMemcpyAsync(offs.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, st),
              "upload");
    hip_check(hipStreamSynchronize(st), "upload");
}

struct Sandwich {
    std::vector<int64_t> in_off, out_off;
    std::vector<int32_t> in_stride, out_stride, a_in, b_in, a_out, b_out, t, s;
    SandwichDev dev{};
    DevMem mem;
    void upload(hipStream_t st)
    {
        Packer pk;
        pk.add(in_off, const_cast<int64_t **>(&dev.in_off));
        pk.add(out_off, const_cast<int64_t **>(&dev.out_off));
        pk.add(in_stride, const_cast<int32_t **>(&dev.in_stride));
        pk.add(out_stride, const_cast<int32_t **>(&dev.out_stride));
        pk.add(a_in, const_cast<int32_t **>(&dev.a_in));
        pk.add(b_in, const_cast<int32_t **>(&dev.b_in));
        pk.add(a_out, const_cast<int32_t **>(&dev.a_out));
        pk.add(b_out, const_cast<int32_t **>(&dev.b_out));
        pk.add(t, const_cast<int32_t **>(&dev.t));
        pk.add(s, const_cast<int32_t **>(&dev.s));
        pk.upload(mem, st);
    }
};

// New coupling panels with the given row/column ranks (groups and segments of
// rank 0 dropped) and the sandwich list mapping the blocks of `in` to them.
void remap_coupling(const RowPanels &in, const Basis &rowb, const Basis &colb,
                    const std::vector<int> &rrank, const std::vector<int> &crank,
                    const std::vector<int64_t> &rhat, const std::vector<int64_t> &chat, RowPanels &out,
                    Sandwich &sw)
{
    (void)rowb;
    (void)colb;
    for (int g = 0; g < in.ngroups(); ++g) {
        const int t = in.group_tag[g];
        if (rrank[t] == 0) continue;
        bool any = false;
        for (int j = in.seg_ptr[g]; j < in.seg_ptr[g + 1]; ++j) any |= crank[in.seg_tag[j]] > 0;
        if (!any) continue;
        out.begin_group(t, (int)rhat[t], rrank[t]);
        struct Pending {
            int64_t in_off;
            int b_in, s, c0;
        };
        std::vector<Pending> pend;
        int cin = 0, cout = 0;
        for (int j = in.seg_ptr[g]; j < in.seg_ptr[g + 1]; ++j) {
            const int s = in.seg_tag[j];
            if (crank[s] > 0) {
                out.add_segment((int)chat[s], crank[s], s);
                pend.push_back({in.val_off[g] + cin, in.seg_len[j], s, cout});
                cout += crank[s];
            }
            cin += in.seg_len[j];
        }
        out.end_group();
        const int gi = out.ngroups() - 1;
        for (auto &p : pend) {
            sw.in_off.push_back(p.in_off);
            sw.in_stride.push_back(in.ncols[g]);
            sw.a_in.push_back(in.nrows[g]);
            sw.b_in.push_back(p.b_in);
            sw.out_off.push_back(out.val_off[gi] + p.c0);
            sw.out_stride.push_back(out.ncols[gi]);
            sw.a_out.push_back(rrank[t]);
            sw.b_out.push_back(crank[p.s]);
            sw.t.push_back(t);
            sw.s.push_back(p.s);
        }
    }
}

template <typename TO>
void run_sandwich(Sandwich &sw, const double *in, TO *out, const DevMem &L, const DevMem &Loff,
                  const DevMem &R, const DevMem &Roff, hipStream_t st)
{
    if (sw.t.empty()) return;
    sw.upload(st);
    const int64_t n = (int64_t)sw.t.size();
    int big = 0;
    for (int64_t b = 0; b < n; ++b)
        big = std::max({big, sw.a_in[b], sw.b_in[b], sw.a_out[b], sw.b_out[b]});
    if (big > RK) {
        if (!std::is_same<TO, double>::value)
            fail(H2B_ENOTSUP, "recompression of ranks above 64 needs an FP64 far field");
        const int tiles = (std::max(*std::max_element(sw.a_out.begin(), sw.a_out.end()),
                                    *std::max_element(sw.b_out.begin(), sw.b_out.end())) + RK - 1) / RK;
        if (n * tiles * tiles >= (int64_t)1 << 31) fail(H2B_ENOTSUP, "too many coupling blocks for one launch");
        hipLaunchKernelGGL(k_sandwich_tiled, dim3((unsigned)(n * tiles * tiles)), dim3(NT), 0, st, sw.dev, tiles, in,
                           reinterpret_cast<double *>(out), L.as<double>(), Loff.as<int64_t>(), R.as<double>(),
                           Roff.as<int64_t>());
        hip_check(hipGetLastError(), "sandwich launch");
        return;
    }
    for (int64_t b0 = 0; b0 < n; b0 += (1 << 30)) {
        // one launch covers every block (n < 2^31 blocks)
        hipLaunchKernelGGL(k_sandwich<TO>, dim3((unsigned)std::min<int64_t>(n - b0, 1 << 30)), dim3(NT), 0,
                           st, sw.dev, in, out, L.as<double>(), Loff.as<int64_t>(), R.as<double>(),
                           Roff.as<int64_t>());
        hip_check(hipGetLastError(), "sandwich launch");
    }
}

void set_basis_values(Basis &B, const Ortho &o, h2b_dtype dt, hipStream_t st)
{
    const Tree &T = *B.tree;
    std::vector<double> leaf(std::max<int64_t>(B.leaf.total, 1)), tr(std::max<int64_t>(B.trans.total, 1));
    for (int g = 0; g < B.leaf.ngroups(); ++g) {
        const int c = B.leaf.group_tag[g];
        std::copy(o.newleaf[c].begin(), o.newleaf[c].end(), leaf.begin() + B.leaf.val_off[g]);
    }
    for (int g = 0; g < B.trans.ngroups(); ++g) {
        const int c = B.trans.group_tag[g];
        std::copy(o.newtr[c].begin(), o.newtr[c].end(), tr.begin() + B.trans.val_off[g]);
    }
    (void)T;
    auto up = [&](const std::vector<double> &v, DevMem &mem) {
        if (dt == H2B_F64) {
            mem.alloc(v.size() * sizeof(double));
            hip_check(hipMemcpyAsync(mem.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st),
                      "upload");
        } else {
            std::vector<float> f(v.begin(), v.end());
            mem.alloc(f.size() * sizeof(float));
            hip_check(hipMemcpyAsync(mem.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st),
                      "upload");
        }
        hip_check(hipStreamSynchronize(st), "upload");
    };
    up(leaf, B.leaf_vals);
    up(tr, B.trans_vals);
}

}  // namespace

void recompress_op(Op &op, double tol, hipStream_t st)
{
    const int m = op.params.order_m;
    const int k = m * m * m;
    const bool shared = (op.colb == op.rowb);
    std::vector<Basis *> bases{op.rowb.get()};
    if (!shared) bases.push_back(op.colb.get());
    std::vector<Ortho> orth(bases.size());

    // 1. orthogonalise (leaf and transfer values from the device)
    for (size_t bi = 0; bi < bases.size(); ++bi) {
        Basis &B = *bases[bi];
        std::vector<double> leafT(std::max<int64_t>(B.leaf.total, 1)), trT(std::max<int64_t>(B.trans.total, 1));
        hip_check(hipMemcpy(leafT.data(), B.leaf_vals.p, sizeof(double) * B.leaf.total, hipMemcpyDeviceToHost),
                  "leaf download");
        if (B.trans.total > 0)
            hip_check(hipMemcpy(trT.data(), B.trans_vals.p, sizeof(double) * B.trans.total, hipMemcpyDeviceToHost),
                      "transfer download");
        orthogonalise(B, leafT, trT, orth[bi]);
    }
    Ortho &orow = orth[0];
    Ortho &ocol = shared ? orth[0] : orth[1];

    // 2. S~ = R_t S R_s^T on the device
    const Tree &Rt = *op.rowb->tree, &Ct = *op.colb->tree;
    std::vector<int64_t> rhat0(Rt.nclusters() + 1, 0), chat0(Ct.nclusters() + 1, 0);
    for (int64_t c = 0; c < Rt.nclusters(); ++c) rhat0[c + 1] = rhat0[c] + orow.r[c];
    for (int64_t c = 0; c < Ct.nclusters(); ++c) chat0[c + 1] = chat0[c] + ocol.r[c];
    RowPanels cplO;
    Sandwich sw1;
    remap_coupling(op.cpl, *op.rowb, *op.colb, orow.r, ocol.r, rhat0, chat0, cplO, sw1);
    DevMem Rr, Rro, Rc, Rco;
    upload_blocks(orow.R, Rr, Rro, st);
    if (!shared) upload_blocks(ocol.R, Rc, Rco, st);
    DevMem stil;
    stil.alloc(sizeof(double) * std::max<int64_t>(cplO.total, 1));
    run_sandwich<double>(sw1, op.cpl_vals.as<double>(), stil.as<double>(), Rr, Rro, shared ? Rr : Rc,
                         shared ? Rro : Rco, st);
    hip_check(hipStreamSynchronize(st), "coupling orthogonalisation");
    op.cpl_vals.release();

    // 3. weights: Gram sums on the device, recursion on the host
    cplO.upload(st);
    ColPanels cplOT;
    transpose_panels(cplO, 0, cplO.ngroups(), cplOT);
    cplOT.upload(st);
    auto gram_offsets = [](const Ortho &o, std::vector<int64_t> &off) {
        off.assign(o.r.size() + 1, 0);
        for (size_t c = 0; c < o.r.size(); ++c) off[c + 1] = off[c] + (int64_t)o.r[c] * o.r[c];
    };
    std::vector<int64_t> grow, gcol;
    gram_offsets(orow, grow);
    gram_offsets(ocol, gcol);
    DevMem dgr, dgro, dgc, dgco, dtag;
    dgr.alloc(sizeof(double) * std::max<int64_t>(grow.back(), 1));
    dgc.alloc(sizeof(double) * std::max<int64_t>(gcol.back(), 1));
    hip_check(hipMemsetAsync(dgr.p, 0, dgr.bytes, st), "memset");
    hip_check(hipMemsetAsync(dgc.p, 0, dgc.bytes, st), "memset");
    dgro.alloc(sizeof(int64_t) * grow.size());
    dgco.alloc(sizeof(int64_t) * gcol.size());
    hip_check(hipMemcpyAsync(dgro.p, grow.data(), sizeof(int64_t) * grow.size(), hipMemcpyHostToDevice, st),
              "upload");
    hip_check(hipMemcpyAsync(dgco.p, gcol.data(), sizeof(int64_t) * gcol.size(), hipMemcpyHostToDevice, st),
              "upload");
    // column-group tags: the column cluster whose coefficients start at out_begin
    std::vector<int32_t> ctag(cplOT.ngroups());
    {
        std::vector<int32_t> by_off(chat0.back() + 1, -1);
        for (int64_t c = Ct.nclusters() - 1; c >= 0; --c)
            if (ocol.r[c] > 0) by_off[chat0[c]] = (int32_t)c;
        for (int g = 0; g < cplOT.ngroups(); ++g) ctag[g] = by_off[cplOT.out_begin[g]];
    }
    dtag.alloc(sizeof(int32_t) * std::max<size_t>(ctag.size(), 1));
    hip_check(hipMemcpyAsync(dtag.p, ctag.data(), sizeof(int32_t) * ctag.size(), hipMemcpyHostToDevice, st),
              "upload");
    if (cplO.ngroups() > 0) {
        const int tr = (cplO.max_nrows + RK - 1) / RK, tc = (cplOT.max_out + RK - 1) / RK;
        if ((int64_t)cplO.ngroups() * tr * tr >= (int64_t)1 << 31 || (int64_t)cplOT.ngroups() * tc * tc >= (int64_t)1 << 31)
            fail(H2B_ENOTSUP, "too many coupling groups for one launch");
        if (tr <= 1)
            hipLaunchKernelGGL(k_gram_rows, dim3(cplO.ngroups()), dim3(NT), 0, st, cplO.dev, stil.as<double>(),
                               dgr.as<double>(), dgro.as<int64_t>());
        else
            hipLaunchKernelGGL(k_gram_rows_tiled, dim3(cplO.ngroups() * tr * tr), dim3(NT), 0, st, cplO.dev, tr,
                               stil.as<double>(), dgr.as<double>(), dgro.as<int64_t>());
        hip_check(hipGetLastError(), "gram launch");
        if (tc <= 1)
            hipLaunchKernelGGL(k_gram_cols, dim3(cplOT.ngroups()), dim3(NT), 0, st, cplOT.dev, stil.as<double>(),
                               dgc.as<double>(), dgco.as<int64_t>(), dtag.as<int32_t>());
        else
            hipLaunchKernelGGL(k_gram_cols_tiled, dim3(cplOT.ngroups() * tc * tc), dim3(NT), 0, st, cplOT.dev, tc,
                               stil.as<double>(), dgc.as<double>(), dgco.as<int64_t>(), dtag.as<int32_t>());
        hip_check(hipGetLastError(), "gram launch");
    }
    std::vector<double> hgr(grow.back()), hgc(gcol.back());
    hip_check(hipMemcpyAsync(hgr.data(), dgr.p, sizeof(double) * hgr.size(), hipMemcpyDeviceToHost, st),
              "download");
    hip_check(hipMemcpyAsync(hgc.data(), dgc.p, sizeof(double) * hgc.size(), hipMemcpyDeviceToHost, st),
              "download");
    hip_check(hipStreamSynchronize(st), "gram");
    orow.Z.assign(Rt.nclusters(), {});
    for (int64_t c = 0; c < Rt.nclusters(); ++c)
        orow.Z[c].assign(hgr.begin() + grow[c], hgr.begin() + grow[c + 1]);
    if (shared) {
        for (int64_t c = 0; c < Rt.nclusters(); ++c)
            for (int64_t i = 0; i < grow[c + 1] - grow[c]; ++i) orow.Z[c][i] += hgc[gcol[c] + i];
    } else {
        ocol.Z.assign(Ct.nclusters(), {});
        for (int64_t c = 0; c < Ct.nclusters(); ++c)
            ocol.Z[c].assign(hgc.begin() + gcol[c], hgc.begin() + gcol[c + 1]);
    }
    for (size_t bi = 0; bi < bases.size(); ++bi) propagate_weights(*bases[bi]->tree, orth[bi]);

    // 4. truncation and new bases
    for (size_t bi = 0; bi < bases.size(); ++bi) {
        truncate_basis(*bases[bi]->tree, tol, orth[bi]);
        Basis &B = *bases[bi];
        B.leaf = RowPanels();
        B.leaf_T = ColPanels();
        B.trans = RowPanels();
        B.trans_T = ColPanels();
        B.leaf_F = ColPanels();
        B.trans_F = ColPanels();
        build_basis_structure(B, orth[bi].kk, st);
        B.leaf.upload(st);
        B.leaf_T.upload(st);
        B.trans.upload(st);
        B.trans_T.upload(st);
        set_basis_values(B, orth[bi], op.params.farfield_dtype, st);
        transpose_basis_values(B, op.params.farfield_dtype, st);
    }

    if (op.recompute) {
        // couplings evaluated on the fly: keep the rank-k block structure
        // (cluster c's interpolation coefficients at c * k) and store the
        // projections P_c = B_c R_c onto the interpolation bases instead
        for (size_t bi = 0; bi < bases.size(); ++bi) {
            const Ortho &o = orth[bi];
            std::vector<std::vector<double>> P(o.kk.size());
            parallel_for((int64_t)o.kk.size(), [&](int64_t c) {
                P[c].assign((size_t)o.kk[c] * k, 0.0);
                if (o.kk[c] > 0) gemm_nn(o.kk[c], k, o.r[c], o.B[c].data(), o.R[c].data(), P[c].data());
            });
            set_projection(*bases[bi], k, P, st);
        }
        return;
    }

    // 5. S'' = B_t S~ B_s^T
    RowPanels cplN;
    Sandwich sw2;
    remap_coupling(cplO, *op.rowb, *op.colb, orow.kk, ocol.kk, op.rowb->hat_off, op.colb->hat_off, cplN,
                   sw2);
    // the input offsets of sw2 refer to cplO, whose groups may be a superset
    DevMem Br, Bro, Bc, Bco;
    upload_blocks(orow.B, Br, Bro, st);
    if (!shared) upload_blocks(ocol.B, Bc, Bco, st);
    DevMem snew;
    snew.alloc(coupling_size(op.params.farfield_dtype) * std::max<int64_t>(cplN.total, 1));
    const DevMem &BcU = shared ? Br : Bc, &BcoU = shared ? Bro : Bco;
    if (op.params.farfield_dtype == H2B_F64)
        run_sandwich<double>(sw2, stil.as<double>(), snew.as<double>(), Br, Bro, BcU, BcoU, st);
    else if (op.params.farfield_dtype == H2B_F32)
        run_sandwich<float>(sw2, stil.as<double>(), snew.as<float>(), Br, Bro, BcU, BcoU, st);
    else
        run_sandwich<bf16_t>(sw2, stil.as<double>(), snew.as<bf16_t>(), Br, Bro, BcU, BcoU, st);
    hip_check(hipStreamSynchronize(st), "coupling projection");
    op.cpl = std::move(cplN);
    op.cpl_T = ColPanels();
    transpose_panels(op.cpl, 0, op.cpl.ngroups(), op.cpl_T);
    op.cpl.upload(st);
    op.cpl_T.upload(st);
    op.cpl_vals = std::move(snew);
}

}  // namespace h2b
