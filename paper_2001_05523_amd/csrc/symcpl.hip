// Far field of G stored once per pair of clusters.
//
// G's kernel is symmetric and G uses one cluster basis for rows and columns,
// so its coupling matrices satisfy S_st = S_ts^T: with interpolation both are
// g at the same pairs of interpolation points (Section 2, eq. (vsw)); with the
// cross approximation both hold G's entries between the same pivot triangles
// of two admissible clusters (Section 4), whose quadrature sums the same
// terms; after recompression both are projected onto the same bases, so the
// equality holds to rounding.  For every row
// cluster t the panel [S_ts for the farfield clusters s > t] is stored; one
// pass (k_cplsym) reads each block once for the row sums y^_t += S_ts x^_s
// and the column sums S_ts^T x^_t, which go to a scratch vector, and a
// second launch (k_cplreduce) adds the column sums per cluster s.  The
// single-vector products G x and G^T x both use it (the far field of G is
// symmetric); the result equals the full coupling product to rounding.  FP64
// and FP32 far fields (values, coefficients and sums in that precision).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <unordered_set>

#include "device.hpp"
#include "op.hpp"

namespace h2b {

namespace {

constexpr int CS_MAXSEG = 256;  // segment descriptors held in LDS
constexpr int CS_NB = 4;        // column blocks of 64 per pass (256 columns)
constexpr int CS_RW = 4;        // rows per step

template <typename T> __device__ inline T wave_sum_c(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// One wave per stored row cluster t (rank at most SYMCPL_MAX_RANK).  A pass
// covers 256 panel columns, one per lane and column block; the inputs x^_s of its columns
// are gathered once (segment by binary search) and the column sums stay in
// registers.  Each step loads 4 rows of the pass (4 x 4 non-temporal loads in
// flight; blocks past the panel's end are skipped for the whole wave, the
// ragged tail is clamped to the last column with weight 0), adds them into the
// row sums (one wave reduction per row) and, weighted with x^_t of the rows,
// into the column sums.  Rows past the end repeat the last row with weight 0.
template <typename T>
__global__ __launch_bounds__(64) void k_cplsym(RowPanelDev d, const T *__restrict__ vals,
                                               const T *__restrict__ xhat, T *__restrict__ yhat,
                                               T *__restrict__ colsum, const int64_t *__restrict__ col_base)
{
    __shared__ T xt[SYMCPL_MAX_RANK + CS_RW], racc[SYMCPL_MAX_RANK];
    __shared__ int32_t lc0[CS_MAXSEG], lin[CS_MAXSEG];
    const int g = blockIdx.x, lane = threadIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int ob = d.out_begin[g];
    const int sb = d.seg_ptr[g], nseg = d.seg_ptr[g + 1] - sb;
    const int32_t *c0s = d.seg_c0 + sb, *ins = d.seg_in + sb;
    if (nseg <= CS_MAXSEG) {
        for (int k = lane; k < nseg; k += 64) {
            lc0[k] = c0s[k];
            lin[k] = ins[k];
        }
        c0s = lc0;
        ins = lin;
    }
    for (int r = lane; r < nr + CS_RW; r += 64) {
        xt[r] = r < nr ? xhat[ob + r] : T(0);  // 0 on the rows past the end
        racc[min(r, SYMCPL_MAX_RANK - 1)] = T(0);
    }
    __syncthreads();
    const int64_t cb = col_base[g];
    const int clast = nc - 1;
    for (int p0 = 0; p0 < nc; p0 += 64 * CS_NB) {
        const int nb = min(CS_NB, (nc - p0 + 63) >> 6);  // column blocks holding columns (uniform)
        T xg[CS_NB], cs[CS_NB];
#pragma unroll
        for (int b = 0; b < CS_NB; ++b) {
            const int c = p0 + lane + 64 * b;
            cs[b] = T(0);
            xg[b] = T(0);
            if (c < nc) {
                int lo = 0, hi = nseg - 1;  // last segment starting at or before c
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (c0s[mid] <= c)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                xg[b] = xhat[ins[lo] + (c - c0s[lo])];
            }
        }
        for (int r = 0; r < nr; r += CS_RW) {
            T a[CS_RW][CS_NB];
#pragma unroll
            for (int i = 0; i < CS_RW; ++i) {
                const T *row = vals + off + (int64_t)min(r + i, nr - 1) * nc;
#pragma unroll
                for (int b = 0; b < CS_NB; ++b)
                    a[i][b] = b < nb ? __builtin_nontemporal_load(row + min(p0 + lane + 64 * b, clast)) : T(0);
            }
            T s[CS_RW];
#pragma unroll
            for (int i = 0; i < CS_RW; ++i) {
                const T w = xt[r + i];  // 0 past the last row
                s[i] = T(0);
#pragma unroll
                for (int b = 0; b < CS_NB; ++b) {
                    s[i] += a[i][b] * xg[b];  // xg is 0 past the last column
                    cs[b] += a[i][b] * w;
                }
            }
#pragma unroll
            for (int i = 0; i < CS_RW; ++i) {
                const T v = wave_sum_c(s[i]);
                if (lane == 0 && r + i < nr) racc[r + i] += v;
            }
        }
#pragma unroll
        for (int b = 0; b < CS_NB; ++b) {
            const int c = p0 + lane + 64 * b;
            if (c < nc) colsum[cb + c] = cs[b];
        }
    }
    __syncthreads();
    for (int r = lane; r < nr; r += 64) yhat[ob + r] += racc[r];
}

// One wave per cluster u: y^_u += the column sums of the stored blocks (t, u),
// in the order of the blocks, 8 loads per batch.
template <typename T>
__global__ __launch_bounds__(64) void k_cplreduce(ColPanelDev red, const T *__restrict__ colsum,
                                                  T *__restrict__ yhat)
{
    const int u = blockIdx.x;
    const int ob = red.out_begin[u], ol = red.out_len[u];
    const int b0 = red.blk_ptr[u], b1 = red.blk_ptr[u + 1];
    for (int j = threadIdx.x; j < ol; j += 64) {
        T acc = T(0);
        for (int b = b0; b < b1; b += 8) {
            T v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const T x = colsum[red.b_val_off[min(b + q, b1 - 1)] + j];
                v[q] = b + q < b1 ? x : T(0);
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) acc += v[q];
        }
        yhat[ob + j] += acc;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_copy_cpl(const int64_t *__restrict__ src_off,
                                                  const int32_t *__restrict__ src_ld,
                                                  const int64_t *__restrict__ dst_off,
                                                  const int32_t *__restrict__ dst_ld,
                                                  const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ cols, const T *__restrict__ src,
                                                  T *__restrict__ dst)
{
    const int b = blockIdx.x;
    const int nr = rows[b], nc = cols[b];
    for (int e = threadIdx.x; e < nr * nc; e += 256) {
        const int r = e / nc, c = e % nc;
        dst[dst_off[b] + (int64_t)r * dst_ld[b] + c] = src[src_off[b] + (int64_t)r * src_ld[b] + c];
    }
}

}  // namespace

void make_symmetric_coupling(Op &op, hipStream_t st)
{
    if (!op.symcpl) {
        const RowPanels &F = op.cpl;
        const Basis &B = *op.rowb;
        const int64_t ncl = B.tree->nclusters();
        auto S = std::make_unique<SymCpl>();
        std::unordered_set<int64_t> blocks;
        for (int g = 0; g < F.ngroups(); ++g)
            for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k)
                blocks.insert((int64_t)F.group_tag[g] * ncl + F.seg_tag[k]);
        std::vector<int> blk_group, blk_c0;
        for (int g = 0; g < F.ngroups(); ++g) {
            const int t = F.group_tag[g];
            bool any = false;
            for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k) any = any || F.seg_tag[k] > t;
            if (!any) continue;
            S->P.begin_group(t, F.out_begin[g], F.nrows[g]);
            for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k) {
                const int s = F.seg_tag[k];
                if (s <= t) continue;
                if (!blocks.count((int64_t)s * ncl + t)) fail(H2B_EINVAL, "farfield blocks are not symmetric");
                S->cp_src.push_back(F.val_off[g] + F.seg_c0[k]);
                S->cp_src_ld.push_back(F.ncols[g]);
                S->cp_rows.push_back(F.nrows[g]);
                S->cp_cols.push_back(F.seg_len[k]);
                blk_group.push_back(S->P.ngroups() - 1);
                blk_c0.push_back(S->P.ncols.back());
                S->P.add_segment(F.seg_in[k], F.seg_len[k], s);
            }
            S->P.end_group();
        }
        if (S->P.max_nrows > SYMCPL_MAX_RANK)
            fail(H2B_ENOTSUP, "the once-per-pair far field needs ranks of at most " + std::to_string(SYMCPL_MAX_RANK));
        for (size_t b = 0; b < blk_group.size(); ++b) {
            S->cp_dst.push_back(S->P.val_off[blk_group[b]] + blk_c0[b]);
            S->cp_dst_ld.push_back(S->P.ncols[blk_group[b]]);
        }
        S->col_base.assign(S->P.ngroups() + 1, 0);
        for (int g = 0; g < S->P.ngroups(); ++g) S->col_base[g + 1] = S->col_base[g] + S->P.ncols[g];
        // per cluster u the column-sum offsets of its stored blocks (t, u), t < u
        std::vector<std::vector<int64_t>> per(ncl);
        for (int g = 0; g < S->P.ngroups(); ++g)
            for (int k = S->P.seg_ptr[g]; k < S->P.seg_ptr[g + 1]; ++k)
                per[S->P.seg_tag[k]].push_back(S->col_base[g] + S->P.seg_c0[k]);
        for (int64_t u = 0; u < ncl; ++u) {
            if (per[u].empty() || B.rank[u] == 0) continue;
            S->red.out_begin.push_back((int32_t)B.hat_off[u]);
            S->red.out_len.push_back(B.rank[u]);
            S->red.max_out = std::max(S->red.max_out, B.rank[u]);
            for (int64_t o : per[u]) S->red.b_val_off.push_back(o);
            S->red.blk_ptr.push_back((int32_t)S->red.b_val_off.size());
        }
        S->P.upload(st);
        S->red.upload(st);
        Packer pk;
        pk.add(S->col_base, const_cast<int64_t **>(&S->d_col_base));
        pk.add(S->cp_src, const_cast<int64_t **>(&S->d_cp_src));
        pk.add(S->cp_dst, const_cast<int64_t **>(&S->d_cp_dst));
        pk.add(S->cp_src_ld, const_cast<int32_t **>(&S->d_cp_src_ld));
        pk.add(S->cp_dst_ld, const_cast<int32_t **>(&S->d_cp_dst_ld));
        pk.add(S->cp_rows, const_cast<int32_t **>(&S->d_cp_rows));
        pk.add(S->cp_cols, const_cast<int32_t **>(&S->d_cp_cols));
        pk.upload(S->desc, st);
        S->f32 = op.params.farfield_dtype == H2B_F32;
        const size_t es = S->f32 ? sizeof(float) : sizeof(double);
        S->vals.alloc(es * std::max<int64_t>(S->P.total, 1));
        S->colsum.alloc(es * std::max<int64_t>(S->col_base.back(), 1));
        S->cp_src.clear();
        S->cp_dst.clear();
        op.symcpl = std::move(S);
    }
    SymCpl &S = *op.symcpl;
    const int nblk = (int)S.cp_rows.size();
    if (nblk > 0 && S.f32)
        hipLaunchKernelGGL(k_copy_cpl<float>, dim3(nblk), dim3(256), 0, st, S.d_cp_src, S.d_cp_src_ld, S.d_cp_dst,
                           S.d_cp_dst_ld, S.d_cp_rows, S.d_cp_cols, op.cpl_vals.as<float>(), S.vals.as<float>());
    else if (nblk > 0)
        hipLaunchKernelGGL(k_copy_cpl<double>, dim3(nblk), dim3(256), 0, st, S.d_cp_src, S.d_cp_src_ld, S.d_cp_dst,
                           S.d_cp_dst_ld, S.d_cp_rows, S.d_cp_cols, op.cpl_vals.as<double>(), S.vals.as<double>());
    hip_check(hipGetLastError(), "coupling copy launch");
    hip_check(hipStreamSynchronize(st), "once-per-pair far field");
}

template <typename T>
void symmetric_coupling_product(const Op &op, const T *xhat, T *yhat, hipStream_t st)
{
    const SymCpl &S = *op.symcpl;
    if (S.f32 != std::is_same<T, float>::value) fail(H2B_EINVAL, "once-per-pair coupling of another precision");
    T *cs = S.colsum.as<T>();
    if (S.P.ngroups() > 0)
        hipLaunchKernelGGL(k_cplsym<T>, dim3(S.P.ngroups()), dim3(64), 0, st, S.P.dev, S.vals.as<T>(), xhat, yhat,
                           cs, S.d_col_base);
    hip_check(hipGetLastError(), "once-per-pair coupling launch");
    if (S.red.ngroups() > 0)
        hipLaunchKernelGGL(k_cplreduce<T>, dim3(S.red.ngroups()), dim3(64), 0, st, S.red.dev, cs, yhat);
    hip_check(hipGetLastError(), "coupling column-sum launch");
}

template void symmetric_coupling_product<double>(const Op &, const double *, double *, hipStream_t);
template void symmetric_coupling_product<float>(const Op &, const float *, float *, hipStream_t);

}  // namespace h2b
