// Forward and backward transformations of a cluster basis, one launch per
// level with one wave per cluster and precomputed work descriptors.
//
// The forward transformation (Section 2, eq. (transfer)) computes the leaf
// coefficients x^_t = V_t^T x|_t and then, up the tree, x^_t = sum over the
// children t' of E_t'^T x^_t'; the backward transformation applies the same
// matrices the other way.  Every level is a launch that waits on memory
// round trips, so what a level costs is the length of one wave's chain of
// dependent loads: reading a cluster's panel descriptor, then its blocks'
// descriptors, then the matrix in small batches.  Here every cluster gets one
// 64-byte descriptor with everything its wave needs (matrix offset, rank, the
// cluster's coefficient offset, its one or two input segments), read at a
// wave-uniform address, and the wave then issues the matrix loads of eight
// rows at once together with its inputs: about two round trips per level.
//
//   forward item:   out[r] = sum_col P[r][col] in(col) with P = V_t^T (a leaf:
//                   columns = the leaf's triangles or vertices) or
//                   [E_c0^T | E_c1^T] (a parent: columns = the children's
//                   coefficients); lanes over columns, wave sums per row;
//   backward item:  out(col) += sum_r P[r][col] y^_t[r], lanes over columns.
//
// Forward order: all leaves, then the parents level by level from the
// deepest; backward: the parents from the root down, then all leaves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <map>

#include "device.hpp"
#include "op.hpp"

namespace h2b {

namespace {

// Descriptor of one cluster (16 int32):
//  [0,1] matrix offset (int64, in the leaf or the transfer value array)
//  [2] rows (the cluster's rank)   [3] the cluster's coefficient offset
//  [4] length, [5] offset of input segment 0   [6] length, [7] offset of segment 1 (0, 0 for leaves)
//  (a leaf's segment: positions in the permuted vector; a parent's: the
//  children's coefficient offsets)
constexpr int DW = 16;
constexpr int RB = 8;  // matrix rows loaded per batch

template <typename T> struct AccT { using type = double; };
template <> struct AccT<float> { using type = float; };

template <typename A> __device__ inline A wave_total(A v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename F, typename XT>
__global__ __launch_bounds__(64) void k_forward_level(const int32_t *__restrict__ desc, int i0,
                                                      const F *__restrict__ vals, const XT *__restrict__ x,
                                                      F *__restrict__ xhat)
{
    using A = typename AccT<F>::type;
    const int32_t *d = desc + (int64_t)(i0 + blockIdx.x) * DW;
    const int64_t voff = (int64_t)(uint32_t)d[0] | ((int64_t)d[1] << 32);
    const int nr = d[2], og = d[3];
    const int len0 = d[4], in0 = d[5], len1 = d[6], in1 = d[7];
    const int nc = len0 + len1;
    const int lane = threadIdx.x;
    const F *P = vals + voff;
    for (int r0 = 0; r0 < nr; r0 += RB) {
        A acc[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = 0;
        for (int c0 = 0; c0 < nc; c0 += 64) {
            const int col = c0 + lane;
            A xin = 0;
            if (col < nc) xin = (A)(col < len0 ? x[in0 + col] : x[in1 + col - len0]);
            const int cc = min(col, nc - 1);
#pragma unroll
            for (int q = 0; q < RB; ++q) acc[q] += (A)P[(int64_t)min(r0 + q, nr - 1) * nc + cc] * xin;
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[q] = wave_total(acc[q]);
        if (lane < RB && r0 + lane < nr) {
            A v = acc[0];
#pragma unroll
            for (int q = 1; q < RB; ++q)
                if (lane == q) v = acc[q];
            xhat[og + r0 + lane] = (F)v;
        }
    }
}

template <typename F, typename YT>
__global__ __launch_bounds__(64) void k_backward_level(const int32_t *__restrict__ desc, int i0,
                                                       const F *__restrict__ vals, const F *__restrict__ yhat_in,
                                                       YT *__restrict__ y)
{
    using A = typename AccT<F>::type;
    const int32_t *d = desc + (int64_t)(i0 + blockIdx.x) * DW;
    const int64_t voff = (int64_t)(uint32_t)d[0] | ((int64_t)d[1] << 32);
    const int nr = d[2], og = d[3];
    const int len0 = d[4], in0 = d[5], len1 = d[6], in1 = d[7];
    const int nc = len0 + len1;
    const int lane = threadIdx.x;
    const F *P = vals + voff;
    const F *par = yhat_in + og;
    for (int c0 = 0; c0 < nc; c0 += 64) {
        const int col = c0 + lane;
        const int cc = min(col, nc - 1);
        A a[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) a[q] = 0;
        for (int r0 = 0; r0 < nr; r0 += RB) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int r = min(r0 + q, nr - 1);
                const A w = r0 + q < nr ? (A)par[r] : A(0);
                a[q] += (A)P[(int64_t)r * nc + cc] * w;
            }
        }
        A v = 0;
#pragma unroll
        for (int q = 0; q < RB; ++q) v += a[q];
        if (col < nc) {
            const int o = col < len0 ? in0 + col : in1 + col - len0;
            y[o] = (YT)((A)y[o] + v);
        }
    }
}

}  // namespace

void build_level_descriptors(Basis &B, hipStream_t st)
{
    const Tree &T = *B.tree;
    const int64_t nc = T.nclusters();
    B.lev = std::make_unique<LevelDescs>();
    LevelDescs &S = *B.lev;
    std::vector<int32_t> leaf_group(nc, -1), trans_group(nc, -1);
    for (int g = 0; g < B.leaf.ngroups(); ++g) leaf_group[B.leaf.group_tag[g]] = g;
    for (int g = 0; g < B.trans.ngroups(); ++g) trans_group[B.trans.group_tag[g]] = g;
    auto descr = [&](int64_t c, std::vector<int32_t> &out) {
        const bool lf = T.nchild[c] == 0;
        const int g = lf ? leaf_group[c] : trans_group[c];
        if (g < 0) fail(H2B_EDEVICE, "a cluster without its basis panel");
        const RowPanels &R = lf ? B.leaf : B.trans;
        const int nseg = R.seg_ptr[g + 1] - R.seg_ptr[g];
        if (nseg != (lf ? 1 : 2) || R.nrows[g] != B.rank[c]) fail(H2B_EDEVICE, "a basis panel of unexpected shape");
        const int64_t vo = R.val_off[g];
        std::vector<int32_t> d(DW, 0);
        d[0] = (int32_t)(uint32_t)(vo & 0xffffffffll);
        d[1] = (int32_t)(vo >> 32);
        d[2] = B.rank[c];
        d[3] = (int32_t)B.hat_off[c];
        for (int s = 0; s < nseg; ++s) {
            const int q = R.seg_ptr[g] + s;
            d[4 + 2 * s] = R.seg_len[q];
            d[5 + 2 * s] = R.seg_in[q];
        }
        // bounds of every address the kernels form from this descriptor
        const int64_t ncol = (int64_t)d[4] + d[6];
        const int64_t lim = lf ? T.n : B.hat_total;
        const bool ok = vo >= 0 && vo + (int64_t)d[2] * ncol <= R.total && d[3] >= 0 && d[3] + d[2] <= B.hat_total &&
                        d[5] >= 0 && d[5] + d[4] <= lim && d[7] >= 0 && d[7] + d[6] <= lim && ncol == R.ncols[g];
        if (!ok) fail(H2B_EDEVICE, "a basis descriptor out of bounds");
        out.insert(out.end(), d.begin(), d.end());
    };
    // forward: the leaves, then the parents by level from the deepest
    std::map<int, std::vector<int64_t>, std::greater<int>> parents;
    std::vector<int64_t> leaves;
    for (int64_t c = 0; c < nc; ++c) {
        if (B.rank[c] == 0) continue;
        if (T.nchild[c] == 0)
            leaves.push_back(c);
        else
            parents[T.level[c]].push_back(c);
    }
    S.step.push_back(0);
    for (int64_t c : leaves) descr(c, S.desc);
    S.step.push_back((int32_t)(S.desc.size() / DW));
    for (auto &kv : parents) {
        for (int64_t c : kv.second) descr(c, S.desc);
        S.step.push_back((int32_t)(S.desc.size() / DW));
    }
    Packer pk;
    pk.add(S.desc, const_cast<int32_t **>(&S.d_desc));
    pk.upload(S.mem, st);
}

template <typename F>
void forward_levels(const Basis &B, const double *xp, F *xhat, hipStream_t st)
{
    const LevelDescs &S = *B.lev;
    for (size_t k = 0; k + 1 < S.step.size(); ++k) {
        const int i0 = S.step[k], n = S.step[k + 1] - i0;
        if (n == 0) continue;
        if (k == 0)
            hipLaunchKernelGGL((k_forward_level<F, double>), dim3(n), dim3(64), 0, st, S.d_desc, i0,
                               B.leaf_vals.as<F>(), xp, xhat);
        else
            hipLaunchKernelGGL((k_forward_level<F, F>), dim3(n), dim3(64), 0, st, S.d_desc, i0, B.trans_vals.as<F>(),
                               (const F *)xhat, xhat);
        hip_check(hipGetLastError(), "forward level launch");
    }
}

template <typename F>
void backward_levels(const Basis &B, F *yhat, double *yp, hipStream_t st)
{
    const LevelDescs &S = *B.lev;
    for (size_t k = S.step.size() - 1; k-- > 0;) {
        const int i0 = S.step[k], n = S.step[k + 1] - i0;
        if (n == 0) continue;
        if (k == 0)
            hipLaunchKernelGGL((k_backward_level<F, double>), dim3(n), dim3(64), 0, st, S.d_desc, i0,
                               B.leaf_vals.as<F>(), (const F *)yhat, yp);
        else
            hipLaunchKernelGGL((k_backward_level<F, F>), dim3(n), dim3(64), 0, st, S.d_desc, i0, B.trans_vals.as<F>(),
                               (const F *)yhat, yhat);
        hip_check(hipGetLastError(), "backward level launch");
    }
}

template void forward_levels<double>(const Basis &, const double *, double *, hipStream_t);
template void forward_levels<float>(const Basis &, const double *, float *, hipStream_t);
template void backward_levels<double>(const Basis &, double *, double *, hipStream_t);
template void backward_levels<float>(const Basis &, float *, double *, hipStream_t);

}  // namespace h2b
