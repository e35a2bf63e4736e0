// Nearfield of the single-layer matrix G on one cluster tree, stored once per
// pair of nearfield leaves.
//
// g(x, y) = g(y, x) makes G symmetric (Section 1, eq. (slp)).  The
// regularised quadrature (Section 5) keeps that exactly, up to rounding, for
// pairs of triangles without a common point: both orders evaluate the same
// tensor Gauss rule.  For touching pairs the two orders of the
// Sauter-Schwab-Erichsen rule agree only to quadrature error.  So the
// product keeps, for every row leaf t, the panel [N_tt | N_ts for s > t], reads
// every off-diagonal block once for y_t += N_ts x_s and y_s += N_ts^T x_t, and
// adds the sparse difference G_ji - G_ij of the touching pairs across leaves,
// which makes the result equal to the full nearfield product.
//
// Launches of one product: k_nearsym (rows: y_t; columns: one sum per panel
// column into a column-sum vector), then k_symreduce (per leaf u: the column sums
// of the blocks (t, u), t != u, plus the corrections of u's rows).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <unordered_map>

#include "device.hpp"
#include "op.hpp"

namespace h2b {
namespace {

constexpr int SYM_NW = 4;         // waves per workgroup of k_nearsym
constexpr int SYM_MAXSEG = 256;   // segment descriptors held in LDS
constexpr int SYM_CHUNK = 2048;   // largest column chunk staged in LDS

__device__ inline double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int find_seg(const int32_t *c0, int n, int col)
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

// One workgroup of 4 waves per row leaf t.  Input columns are gathered into
// LDS (x of the column segments; for G^T x the diagonal columns are set to 0,
// because the diagonal block enters transposed, through its column sums).
// Each wave streams two rows at a time with coalesced non-temporal loads, 4
// column blocks of 64 per step and the last < 4 blocks issued together under
// per-lane predicates; the products feed the row sums (wave reductions) and,
// weighted by x_t of the two rows, the column sums in LDS (ds_add_f64).
// Column sums of the diagonal block go to y_t for G^T x and are dropped for
// G x; the others go to the column-sum vector.
template <bool TRANS>
__global__ __launch_bounds__(SYM_NW * 64) void k_nearsym(RowPanelDev d, int chunk, const double *__restrict__ vals,
                                                         const double *__restrict__ x, double *__restrict__ y,
                                                         double *__restrict__ colsum,
                                                         const int64_t *__restrict__ col_base)
{
    constexpr int NTH = SYM_NW * 64;
    constexpr int NB = 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *xs = reinterpret_cast<double *>(smem_raw);  // chunk
    double *cs = xs + chunk;                            // chunk
    double *racc = cs + chunk;                          // rows
    __shared__ double xt[64];
    __shared__ int32_t lds_c0[SYM_MAXSEG], lds_in[SYM_MAXSEG];
    const int g = blockIdx.x;
    const int nr = d.nrows[g], nc = d.ncols[g];
    const int64_t off = d.val_off[g];
    const int ob = d.out_begin[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sb = d.seg_ptr[g], nseg = d.seg_ptr[g + 1] - sb;
    const int ndiag = d.seg_len[sb];
    const int32_t *c0s = d.seg_c0 + sb, *ins = d.seg_in + sb;
    if (nseg <= SYM_MAXSEG) {
        for (int t = threadIdx.x; t < nseg; t += NTH) {
            lds_c0[t] = c0s[t];
            lds_in[t] = ins[t];
        }
        c0s = lds_c0;
        ins = lds_in;
    }
    for (int i = threadIdx.x; i < nr; i += NTH) xt[i] = x[ob + i];
    __syncthreads();

    for (int c0 = 0; c0 < nc; c0 += chunk) {
        const int clen = min(chunk, nc - c0);
        for (int e0 = threadIdx.x; e0 < clen; e0 += 8 * NTH) {
            double v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * NTH;
                const int col = c0 + e;
                v[q] = 0;
                if (e < clen && !(TRANS && col < ndiag)) {
                    const int sg = find_seg(c0s, nseg, col);
                    v[q] = x[ins[sg] + (col - c0s[sg])];
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int e = e0 + q * NTH;
                if (e < clen) {
                    xs[e] = v[q];
                    cs[e] = 0;
                }
            }
        }
        __syncthreads();
        for (int r = 2 * wave; r < nr; r += 2 * SYM_NW) {
            const bool two = r + 1 < nr;
            const double *row0 = vals + off + (int64_t)r * nc + c0;
            const double *row1 = two ? row0 + nc : row0;
            const double w0 = xt[r], w1 = two ? xt[r + 1] : 0.0;
            double a[NB] = {0, 0, 0, 0}, b[NB] = {0, 0, 0, 0};
            int c = lane;
            for (; c + 64 * (NB - 1) < clen; c += 64 * NB) {
                double p[NB], q[NB];
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    p[k] = __builtin_nontemporal_load(row0 + c + 64 * k);
                    q[k] = __builtin_nontemporal_load(row1 + c + 64 * k);
                }
#pragma unroll
                for (int k = 0; k < NB; ++k) {
                    const double xv = xs[c + 64 * k];
                    a[k] += p[k] * xv;
                    b[k] += q[k] * xv;
                    atomicAdd(&cs[c + 64 * k], p[k] * w0 + q[k] * w1);
                }
            }
            if (c < clen) {  // fewer than NB blocks left
                double p[NB - 1], q[NB - 1];
#pragma unroll
                for (int k = 0; k < NB - 1; ++k) {
                    const bool in = c + 64 * k < clen;
                    p[k] = in ? __builtin_nontemporal_load(row0 + c + 64 * k) : 0.0;
                    q[k] = in ? __builtin_nontemporal_load(row1 + c + 64 * k) : 0.0;
                }
#pragma unroll
                for (int k = 0; k < NB - 1; ++k) {
                    if (c + 64 * k < clen) {
                        const double xv = xs[c + 64 * k];
                        a[k] += p[k] * xv;
                        b[k] += q[k] * xv;
                        atomicAdd(&cs[c + 64 * k], p[k] * w0 + q[k] * w1);
                    }
                }
            }
            const double sa = wave_sum_d((a[0] + a[1]) + (a[2] + a[3]));
            const double sbv = wave_sum_d((b[0] + b[1]) + (b[2] + b[3]));
            if (lane == 0) {
                racc[r] = (c0 == 0) ? sa : racc[r] + sa;
                if (two) racc[r + 1] = (c0 == 0) ? sbv : racc[r + 1] + sbv;
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < clen; e += NTH) {
            const int col = c0 + e;
            if (col >= ndiag)
                colsum[col_base[g] + col] = cs[e];
            else if (TRANS)
                racc[col] += cs[e];  // diagonal column col is row col of t
        }
        __syncthreads();
    }
    for (int r = threadIdx.x; r < nr; r += NTH) y[ob + r] += (nc > 0) ? racc[r] : 0.0;
}

// One wave per leaf u: y_u += sum of the column sums of the blocks (t, u),
// t != u, plus the corrections of u's rows (CSR over cluster-ordered rows).
// Both lists go in batches of 8 loads (the last batch clamped and weighted 0).
__global__ __launch_bounds__(64) void k_symreduce(ColPanelDev red, const double *__restrict__ colsum,
                                                  const int64_t *__restrict__ cptr,
                                                  const int32_t *__restrict__ cidx,
                                                  const double *__restrict__ cval, const double *__restrict__ x,
                                                  double *__restrict__ y)
{
    const int u = blockIdx.x;
    const int ob = red.out_begin[u], ol = red.out_len[u];
    const int b0 = red.blk_ptr[u], b1 = red.blk_ptr[u + 1];
    for (int j = threadIdx.x; j < ol; j += 64) {
        double acc = 0;
        for (int b = b0; b < b1; b += 8) {
            double a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double v = colsum[red.b_val_off[min(b + q, b1 - 1)] + j];
                a[q] = (b + q < b1) ? v : 0.0;
            }
            acc += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
        const int row = ob + j;
        const int64_t e0 = cptr[row], e1 = cptr[row + 1];
        for (int64_t e = e0; e < e1; e += 8) {
            double a[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int64_t ee = min(e + q, e1 - 1);
                const double v = cval[ee] * x[cidx[ee]];
                a[q] = (e + q < e1) ? v : 0.0;
            }
            acc += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
        y[row] += acc;
    }
}

// Copies rows x cols blocks between row-major panels.
__global__ __launch_bounds__(256) void k_copy_blocks(const int64_t *__restrict__ src_off,
                                                     const int32_t *__restrict__ src_ld,
                                                     const int64_t *__restrict__ dst_off,
                                                     const int32_t *__restrict__ dst_ld,
                                                     const int32_t *__restrict__ rows,
                                                     const int32_t *__restrict__ cols,
                                                     const double *__restrict__ src, double *__restrict__ dst)
{
    const int b = blockIdx.x;
    const int nr = rows[b], nc = cols[b];
    for (int e = threadIdx.x; e < nr * nc; e += 256) {
        const int r = e / nc, c = e % nc;
        dst[dst_off[b] + (int64_t)r * dst_ld[b] + c] = src[src_off[b] + (int64_t)r * src_ld[b] + c];
    }
}

// out[e] = near[a[e]] - near[b[e]]
__global__ void k_corr_values(int64_t n, const int64_t *__restrict__ a, const int64_t *__restrict__ b,
                              const double *__restrict__ near, double *__restrict__ out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = near[a[e]] - near[b[e]];
}

int grid_of(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + 255) / 256, 1), 1 << 16); }

// Structure of the once-per-pair storage from the full nearfield panels.
void build_structure(const Op &op, SymNear &S)
{
    const Tree &T = *op.blocks->rows;
    const Mesh &M = *T.mesh;
    const RowPanels &F = op.near;
    const int64_t ncl = T.nclusters();
    std::vector<int> group_of(ncl, -1);
    for (int g = 0; g < F.ngroups(); ++g) group_of[F.group_tag[g]] = g;
    // column of segment (group g, column leaf s) in the full panels
    std::unordered_map<int64_t, int> fc0;
    fc0.reserve(F.seg_in.size() * 2);
    for (int g = 0; g < F.ngroups(); ++g)
        for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k) fc0[(int64_t)g * ncl + F.seg_tag[k]] = F.seg_c0[k];
    auto full_c0 = [&](int g, int s) -> int {
        auto it = fc0.find((int64_t)g * ncl + s);
        if (it == fc0.end()) fail(H2B_EINVAL, "nearfield leaves are not symmetric");
        return it->second;
    };

    // panels [N_tt | N_ts, s > t] and the copy descriptors
    std::vector<int> blk_group, blk_c0;
    for (int g = 0; g < F.ngroups(); ++g) {
        const int t = F.group_tag[g];
        S.P.begin_group(t, F.out_begin[g], F.nrows[g]);
        auto add = [&](int k) {
            S.cp_src.push_back(F.val_off[g] + F.seg_c0[k]);
            S.cp_src_ld.push_back(F.ncols[g]);
            S.cp_rows.push_back(F.nrows[g]);
            S.cp_cols.push_back(F.seg_len[k]);
            blk_group.push_back(g);
            blk_c0.push_back(S.P.ncols.back());
            S.P.add_segment(F.seg_in[k], F.seg_len[k], F.seg_tag[k]);
        };
        int kd = -1;
        for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k)
            if (F.seg_tag[k] == t) kd = k;
        if (kd < 0) fail(H2B_EINVAL, "nearfield leaf without its diagonal block");
        add(kd);
        for (int k = F.seg_ptr[g]; k < F.seg_ptr[g + 1]; ++k)
            if (F.seg_tag[k] > t) {
                (void)full_c0(group_of[F.seg_tag[k]], t);  // the mirror block exists
                add(k);
            }
        S.P.end_group();
    }
    if (S.P.max_nrows > 64) fail(H2B_ENOTSUP, "the once-per-pair nearfield needs leaves of at most 64");
    for (size_t b = 0; b < blk_group.size(); ++b) {
        const int g = blk_group[b];
        S.cp_dst.push_back(S.P.val_off[g] + blk_c0[b]);
        S.cp_dst_ld.push_back(S.P.ncols[g]);
    }
    S.col_base.resize(S.P.ngroups() + 1, 0);
    for (int g = 0; g < S.P.ngroups(); ++g) S.col_base[g + 1] = S.col_base[g] + S.P.ncols[g];

    // reduction lists: per leaf u (group order) the column-sum offsets of (t, u), t != u
    std::vector<std::vector<int64_t>> per_leaf(ncl);
    for (int g = 0; g < S.P.ngroups(); ++g)
        for (int k = S.P.seg_ptr[g] + 1; k < S.P.seg_ptr[g + 1]; ++k)
            per_leaf[S.P.seg_tag[k]].push_back(S.col_base[g] + S.P.seg_c0[k]);
    for (int g = 0; g < F.ngroups(); ++g) {
        const int u = F.group_tag[g];
        S.red.out_begin.push_back(T.begin[u]);
        S.red.out_len.push_back(T.size(u));
        S.red.max_out = std::max(S.red.max_out, T.size(u));
        for (int64_t o : per_leaf[u]) {
            S.red.b_val_off.push_back(o);
            S.red.b_stride.push_back(0);
            S.red.b_c0.push_back(0);
            S.red.b_nrows.push_back(0);
            S.red.b_in.push_back(0);
        }
        S.red.blk_ptr.push_back((int32_t)S.red.b_val_off.size());
    }

    // touching pairs across leaves (a common vertex), t < s
    const int64_t n = T.n;
    std::vector<int32_t> pos_of(n), leaf_at(n, -1);
    for (int64_t p = 0; p < n; ++p) pos_of[T.perm[p]] = (int32_t)p;
    for (int c : T.leaves)
        for (int p = T.begin[c]; p < T.end[c]; ++p) leaf_at[p] = c;
    struct Corr {
        int32_t row_f, idx_f;  // G x: row p_j, input p_i
        int64_t a, b;
    };
    std::vector<Corr> corr;
    std::vector<int32_t> cand;
    for (int64_t i = 0; i < n; ++i) {
        cand.clear();
        for (int32_t v : {M.t0[i], M.t1[i], M.t2[i]})
            for (int64_t e = M.vt_ptr[v]; e < M.vt_ptr[v + 1]; ++e)
                if (M.vt_idx[e] != i) cand.push_back(M.vt_idx[e]);
        std::sort(cand.begin(), cand.end());
        cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
        const int pi = pos_of[i], t = leaf_at[pi];
        for (int32_t j : cand) {
            const int pj = pos_of[j], s = leaf_at[pj];
            if (!(t < s)) continue;
            const int gt = group_of[t], gs = group_of[s];
            Corr c;
            c.row_f = pj;
            c.idx_f = pi;
            c.a = F.val_off[gs] + (int64_t)(pj - T.begin[s]) * F.ncols[gs] + full_c0(gs, t) + (pi - T.begin[t]);
            c.b = F.val_off[gt] + (int64_t)(pi - T.begin[t]) * F.ncols[gt] + full_c0(gt, s) + (pj - T.begin[s]);
            corr.push_back(c);
        }
    }
    S.ncorr = (int64_t)corr.size();
    auto csr = [&](bool fwd, std::vector<int64_t> &ptr, std::vector<int32_t> &idx, std::vector<int64_t> &a,
                   std::vector<int64_t> &b) {
        ptr.assign(n + 1, 0);
        for (auto &c : corr) ++ptr[(fwd ? c.row_f : c.idx_f) + 1];
        for (int64_t r = 0; r < n; ++r) ptr[r + 1] += ptr[r];
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        idx.resize(corr.size());
        a.resize(corr.size());
        b.resize(corr.size());
        for (auto &c : corr) {
            const int64_t e = fill[fwd ? c.row_f : c.idx_f]++;
            idx[e] = fwd ? c.idx_f : c.row_f;
            a[e] = c.a;
            b[e] = c.b;
        }
    };
    csr(true, S.cf_ptr, S.cf_idx, S.cf_a, S.cf_b);
    csr(false, S.cb_ptr, S.cb_idx, S.cb_a, S.cb_b);
}

}  // namespace

void make_symmetric_near(Op &op, hipStream_t st)
{
    if (!op.sym) {
        auto S = std::make_unique<SymNear>();
        build_structure(op, *S);
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
        pk.add(S->cf_ptr, const_cast<int64_t **>(&S->d_cf_ptr));
        pk.add(S->cf_idx, const_cast<int32_t **>(&S->d_cf_idx));
        pk.add(S->cf_a, const_cast<int64_t **>(&S->d_cf_a));
        pk.add(S->cf_b, const_cast<int64_t **>(&S->d_cf_b));
        pk.add(S->cb_ptr, const_cast<int64_t **>(&S->d_cb_ptr));
        pk.add(S->cb_idx, const_cast<int32_t **>(&S->d_cb_idx));
        pk.add(S->cb_a, const_cast<int64_t **>(&S->d_cb_a));
        pk.add(S->cb_b, const_cast<int64_t **>(&S->d_cb_b));
        pk.upload(S->desc, st);
        S->vals.alloc(sizeof(double) * std::max<int64_t>(S->P.total, 1));
        S->colsum.alloc(sizeof(double) * std::max<int64_t>(S->col_base.back(), 1));
        S->cf_val.alloc(sizeof(double) * std::max<int64_t>(S->ncorr, 1));
        S->cb_val.alloc(sizeof(double) * std::max<int64_t>(S->ncorr, 1));
        // host copies of what the kernels read from the descriptors are no longer needed
        S->cp_src.clear();
        S->cp_dst.clear();
        S->cf_a.clear();
        S->cf_b.clear();
        S->cb_a.clear();
        S->cb_b.clear();
        op.sym = std::move(S);
    }
    SymNear &S = *op.sym;
    const int nblk = (int)S.cp_rows.size();
    if (nblk > 0)
        hipLaunchKernelGGL(k_copy_blocks, dim3(nblk), dim3(256), 0, st, S.d_cp_src, S.d_cp_src_ld, S.d_cp_dst,
                           S.d_cp_dst_ld, S.d_cp_rows, S.d_cp_cols, op.near_vals.as<double>(), S.vals.as<double>());
    hip_check(hipGetLastError(), "block copy launch");
    if (S.ncorr > 0) {
        hipLaunchKernelGGL(k_corr_values, dim3(grid_of(S.ncorr)), dim3(256), 0, st, S.ncorr, S.d_cf_a, S.d_cf_b,
                           op.near_vals.as<double>(), S.cf_val.as<double>());
        hipLaunchKernelGGL(k_corr_values, dim3(grid_of(S.ncorr)), dim3(256), 0, st, S.ncorr, S.d_cb_a, S.d_cb_b,
                           op.near_vals.as<double>(), S.cb_val.as<double>());
    }
    hip_check(hipGetLastError(), "correction launch");
    hip_check(hipStreamSynchronize(st), "once-per-pair nearfield");
}

void symmetric_near_product(const Op &op, int trans, const double *xp, double *ypn, hipStream_t st)
{
    const SymNear &S = *op.sym;
    const int ng = S.P.ngroups();
    if (ng == 0) return;
    const int chunk = std::min(SYM_CHUNK, std::max(64, (S.P.max_ncols + 63) / 64 * 64));
    if (chunk < S.P.max_nrows) fail(H2B_EINVAL, "column chunk smaller than a leaf");
    const size_t shm = sizeof(double) * (2 * (size_t)chunk + 64);
    double *cs = S.colsum.as<double>();
    if (trans)
        hipLaunchKernelGGL(k_nearsym<true>, dim3(ng), dim3(SYM_NW * 64), shm, st, S.P.dev, chunk,
                           S.vals.as<double>(), xp, ypn, cs, S.d_col_base);
    else
        hipLaunchKernelGGL(k_nearsym<false>, dim3(ng), dim3(SYM_NW * 64), shm, st, S.P.dev, chunk,
                           S.vals.as<double>(), xp, ypn, cs, S.d_col_base);
    hip_check(hipGetLastError(), "symmetric nearfield launch");
    hipLaunchKernelGGL(k_symreduce, dim3(S.red.ngroups()), dim3(64), 0, st, S.red.dev, cs,
                       trans ? S.d_cb_ptr : S.d_cf_ptr, trans ? S.d_cb_idx : S.d_cf_idx,
                       trans ? S.cb_val.as<double>() : S.cf_val.as<double>(), xp, ypn);
    hip_check(hipGetLastError(), "column-sum reduction launch");
}

}  // namespace h2b
