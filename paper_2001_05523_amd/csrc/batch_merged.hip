// Batched products with one launch per step for all operators.
//
// A batch of meshes (operators of different sizes) runs the same sequence of
// steps for every operator: gather, leaf forward transformation, the transfer
// levels from the bottom, coupling, the transfer levels from the top, leaf
// backward transformation, nearfield, scatter.  Here the panels of every
// operator for one step are merged into one panel set, so that one launch
// covers the step for the whole batch and fills the GPU even when each mesh
// alone would not.  The merged panels keep pointing at each operator's own
// stored values (offsets relative to the lowest value address of the step);
// the work vectors of all operators are slices of vectors owned by the batch.
// Transfer levels are merged by their distance from the leaves going up and
// from the root going down, which keeps every operator's own order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <type_traits>

#include "op.hpp"

namespace h2b {

namespace {

constexpr int BT = 256;

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + BT - 1) / BT, 1 << 20)); }

// xp[k rb + r] = xbase[src[k] + r ld[k]] for r < nb, 0 for nb <= r < rb.
__global__ __launch_bounds__(BT) void k_gather_abs(const int64_t *__restrict__ src, const int64_t *__restrict__ ld,
                                                   int64_t n, int nb, int rb, const double *__restrict__ xbase,
                                                   double *__restrict__ xp)
{
    const int64_t tot = n * rb;
    for (int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * BT) {
        const int64_t k = e / rb;
        const int r = (int)(e % rb);
        xp[e] = r < nb ? xbase[src[k] + r * ld[k]] : 0.0;
    }
}

// ybase[dst[k] + r ld[k]] += alpha[k] (yp[k rb + r] + ypn[k rb + r]) for r < nb.
__global__ __launch_bounds__(BT) void k_scatter_abs(const int64_t *__restrict__ dst, const int64_t *__restrict__ ld,
                                                    const double *__restrict__ alpha, int64_t n, int nb, int rb,
                                                    const double *__restrict__ yp, const double *__restrict__ ypn,
                                                    double *__restrict__ ybase)
{
    const int64_t tot = n * nb;
    for (int64_t e = blockIdx.x * (int64_t)BT + threadIdx.x; e < tot; e += (int64_t)gridDim.x * BT) {
        const int64_t k = e / nb;
        const int r = (int)(e % nb);
        ybase[dst[k] + r * ld[k]] += alpha[k] * (yp[k * rb + r] + ypn[k * rb + r]);
    }
}

int32_t checked32(int64_t v)
{
    if (v < 0 || v > INT32_MAX) fail(H2B_ENOTSUP, "merged batch offsets exceed 32 bits");
    return (int32_t)v;
}

struct RowSrc {
    const RowPanels *rp;
    int g0, g1;
    const void *vals;
    int64_t out_shift, in_shift;  // added to out_begin and to seg_in
};
struct ColSrc {
    const ColPanels *cp;
    int g0, g1;
    const void *vals;
    int64_t out_shift, in_shift;  // added to out_begin and to b_in
};

const char *lowest(const std::vector<const void *> &ptrs)
{
    const char *base = nullptr;
    for (const void *p : ptrs)
        if (p && (!base || static_cast<const char *>(p) < base)) base = static_cast<const char *>(p);
    return base;
}

template <typename T> const T *merge_rows(const std::vector<RowSrc> &src, RowPanels &out, hipStream_t st)
{
    out = RowPanels();
    std::vector<const void *> ptrs;
    for (auto &s : src)
        if (s.g1 > s.g0) ptrs.push_back(s.vals);
    const char *base = lowest(ptrs);
    for (auto &s : src) {
        if (s.g1 <= s.g0) continue;
        const int64_t vs = (static_cast<const char *>(s.vals) - base) / (int64_t)sizeof(T);
        for (int g = s.g0; g < s.g1; ++g) {
            out.begin_group(s.rp->group_tag[g], checked32(s.rp->out_begin[g] + s.out_shift), s.rp->nrows[g]);
            for (int q = s.rp->seg_ptr[g]; q < s.rp->seg_ptr[g + 1]; ++q)
                out.add_segment(checked32(s.rp->seg_in[q] + s.in_shift), s.rp->seg_len[q], s.rp->seg_tag[q]);
            out.end_group();
            out.val_off.back() = s.rp->val_off[g] + vs;
        }
    }
    out.upload(st);
    return reinterpret_cast<const T *>(base);
}

template <typename T> const T *merge_cols(const std::vector<ColSrc> &src, ColPanels &out, hipStream_t st)
{
    out = ColPanels();
    std::vector<const void *> ptrs;
    for (auto &s : src)
        if (s.g1 > s.g0) ptrs.push_back(s.vals);
    const char *base = lowest(ptrs);
    for (auto &s : src) {
        if (s.g1 <= s.g0) continue;
        const int64_t vs = (static_cast<const char *>(s.vals) - base) / (int64_t)sizeof(T);
        const ColPanels &c = *s.cp;
        for (int g = s.g0; g < s.g1; ++g) {
            out.out_begin.push_back(checked32(c.out_begin[g] + s.out_shift));
            out.out_len.push_back(c.out_len[g]);
            out.out_tag.push_back(c.out_tag.empty() ? 0 : c.out_tag[g]);
            out.max_out = std::max(out.max_out, c.out_len[g]);
            for (int b = c.blk_ptr[g]; b < c.blk_ptr[g + 1]; ++b) {
                out.b_val_off.push_back(c.b_val_off[b] + vs);
                out.b_stride.push_back(c.b_stride[b]);
                out.b_c0.push_back(c.b_c0[b]);
                out.b_nrows.push_back(c.b_nrows[b]);
                out.b_in.push_back(checked32(c.b_in[b] + s.in_shift));
                out.b_tag.push_back(c.b_tag.empty() ? 0 : c.b_tag[b]);
            }
            out.blk_ptr.push_back((int32_t)out.b_in.size());
        }
    }
    out.upload(st);
    return reinterpret_cast<const T *>(base);
}

}  // namespace

// Merged panels of every step and the batch's own work vectors.
struct MergedBatch {
    int rb = 1, nb = 1, trans = 0;
    h2b_dtype dt = H2B_F64;
    int64_t nin = 0, nout = 0, hin = 0, hout = 0;
    DevMem xp, yp, ypn, xhat, yhat, gsrc, gld, sdst, sld, salpha;
    const double *xbase = nullptr;
    double *ybase = nullptr;
    // forward: column products over the transposed copies (one vector) or
    // row panels on matrix cores (blocks)
    ColPanels leafF;
    RowPanels leafIn;
    const void *leafF_v = nullptr, *leafIn_v = nullptr;
    std::vector<ColPanels> transF;
    std::vector<RowPanels> transIn;
    std::vector<const void *> transF_v, transIn_v;
    RowPanels cpl;
    const void *cpl_v = nullptr;
    // backward: transposed row panels (one vector) or column panels (blocks)
    std::vector<RowPanels> transOut;
    std::vector<ColPanels> transOutT;
    std::vector<const void *> transOut_v, transOutT_v;
    RowPanels leafOut;
    ColPanels leafOutT;
    const void *leafOut_v = nullptr, *leafOutT_v = nullptr;
    RowPanels near;
    const double *near_v = nullptr;
};

void MergedBatchDeleter::operator()(MergedBatch *m) const { delete m; }

MergedPtr merged_create(int nops, Op *const *ops, const int *trans, const double *alpha, const double *const *x,
                        const int64_t *ldx, double *const *y, const int64_t *ldy, const int *nrhs, hipStream_t st)
{
    // one program for all operators: same storage type, direction and width
    for (int i = 0; i < nops; ++i) {
        const Op &op = *ops[i];
        if (op.params.farfield_dtype != ops[0]->params.farfield_dtype || trans[i] != trans[0] ||
            nrhs[i] != nrhs[0] || op.recompute || (trans[i] && !op.has_R))
            return MergedPtr();
    }
    MergedPtr m(new MergedBatch);
    m->trans = trans[0] ? 1 : 0;
    m->dt = ops[0]->params.farfield_dtype;
    m->nb = nrhs[0];
    m->rb = m->nb == 1 ? 1 : m->nb <= 16 ? 16 : m->nb <= 32 ? 32 : 64;
    const int rb = m->rb;
    const size_t fsz = basis_size(m->dt), csz = coupling_size(m->dt);
    (void)csz;
    // slices of the work vectors
    std::vector<int64_t> xo(nops), yo(nops), xho(nops), yho(nops);
    std::vector<const void *> xs, ys;
    for (int i = 0; i < nops; ++i) {
        const Op &op = *ops[i];
        const Basis &Bin = m->trans ? *op.rowb : *op.colb, &Bout = m->trans ? *op.colb : *op.rowb;
        xo[i] = m->nin;
        yo[i] = m->nout;
        xho[i] = m->hin;
        yho[i] = m->hout;
        m->nin += Bin.tree->n;
        m->nout += Bout.tree->n;
        m->hin += Bin.hat_total;
        m->hout += Bout.hat_total;
        xs.push_back(x[i]);
        ys.push_back(y[i]);
    }
    m->xbase = reinterpret_cast<const double *>(lowest(xs));
    m->ybase = const_cast<double *>(reinterpret_cast<const double *>(lowest(ys)));
    // gather and scatter tables (element offsets from the lowest vector)
    {
        std::vector<int64_t> src(m->nin), gl(m->nin), dst(m->nout), sl(m->nout);
        std::vector<double> al(m->nout);
        for (int i = 0; i < nops; ++i) {
            const Op &op = *ops[i];
            const Basis &Bin = m->trans ? *op.rowb : *op.colb, &Bout = m->trans ? *op.colb : *op.rowb;
            const int64_t xsh = x[i] - m->xbase, ysh = y[i] - m->ybase;
            for (int64_t k = 0; k < Bin.tree->n; ++k) {
                src[xo[i] + k] = xsh + Bin.tree->perm[k];
                gl[xo[i] + k] = ldx[i];
            }
            for (int64_t k = 0; k < Bout.tree->n; ++k) {
                dst[yo[i] + k] = ysh + Bout.tree->perm[k];
                sl[yo[i] + k] = ldy[i];
                al[yo[i] + k] = alpha[i];
            }
        }
        auto up = [&](DevMem &mem, const void *p, size_t bytes) {
            mem.alloc(bytes);
            hip_check(hipMemcpyAsync(mem.p, p, bytes, hipMemcpyHostToDevice, st), "batch table upload");
        };
        up(m->gsrc, src.data(), sizeof(int64_t) * src.size());
        up(m->gld, gl.data(), sizeof(int64_t) * gl.size());
        up(m->sdst, dst.data(), sizeof(int64_t) * dst.size());
        up(m->sld, sl.data(), sizeof(int64_t) * sl.size());
        up(m->salpha, al.data(), sizeof(double) * al.size());
        hip_check(hipStreamSynchronize(st), "batch table upload");
    }
    m->xp.alloc(sizeof(double) * std::max<int64_t>(m->nin, 1) * rb);
    m->yp.alloc(sizeof(double) * std::max<int64_t>(m->nout, 1) * rb);
    m->ypn.alloc(sizeof(double) * std::max<int64_t>(m->nout, 1) * rb);
    m->xhat.alloc(fsz * std::max<int64_t>(m->hin, 1) * rb);
    m->yhat.alloc(fsz * std::max<int64_t>(m->hout, 1) * rb);

    // merged panels of every step
    const bool dbl = m->dt == H2B_F64;
    auto fb = [&](auto *tag, const std::vector<RowSrc> &s, RowPanels &out) -> const void * {
        using T = std::remove_pointer_t<decltype(tag)>;
        return merge_rows<T>(s, out, st);
    };
    auto fc = [&](auto *tag, const std::vector<ColSrc> &s, ColPanels &out) -> const void * {
        using T = std::remove_pointer_t<decltype(tag)>;
        return merge_cols<T>(s, out, st);
    };
    auto basis_rows = [&](const std::vector<RowSrc> &s, RowPanels &out) {
        return dbl ? fb((double *)nullptr, s, out) : fb((float *)nullptr, s, out);
    };
    auto basis_cols = [&](const std::vector<ColSrc> &s, ColPanels &out) {
        return dbl ? fc((double *)nullptr, s, out) : fc((float *)nullptr, s, out);
    };
    size_t nup = 0, ndown = 0;
    for (int i = 0; i < nops; ++i) {
        const Op &op = *ops[i];
        const Basis &Bin = m->trans ? *op.rowb : *op.colb, &Bout = m->trans ? *op.colb : *op.rowb;
        nup = std::max(nup, Bin.fw_steps.size());
        ndown = std::max(ndown, Bout.fw_steps.size());
    }
    {
        std::vector<ColSrc> lf;
        std::vector<RowSrc> li;
        for (int i = 0; i < nops; ++i) {
            const Basis &Bin = m->trans ? *ops[i]->rowb : *ops[i]->colb;
            lf.push_back({&Bin.leaf_F, 0, Bin.leaf_F.ngroups(), Bin.leafT_vals.p, xho[i], xo[i]});
            li.push_back({&Bin.leaf, 0, Bin.leaf.ngroups(), Bin.leaf_vals.p, xho[i], xo[i]});
        }
        m->leafF_v = basis_cols(lf, m->leafF);
        m->leafIn_v = basis_rows(li, m->leafIn);
    }
    m->transF.resize(nup);
    m->transIn.resize(nup);
    m->transF_v.resize(nup);
    m->transIn_v.resize(nup);
    for (size_t lv = 0; lv < nup; ++lv) {
        std::vector<ColSrc> tf;
        std::vector<RowSrc> ti;
        for (int i = 0; i < nops; ++i) {
            const Basis &Bin = m->trans ? *ops[i]->rowb : *ops[i]->colb;
            if (lv >= Bin.fw_steps.size()) continue;
            const auto &s = Bin.fw_steps[lv];
            tf.push_back({&Bin.trans_F, s.first, s.second, Bin.transT_vals.p, xho[i], xho[i]});
            ti.push_back({&Bin.trans, s.first, s.second, Bin.trans_vals.p, xho[i], xho[i]});
        }
        m->transF_v[lv] = basis_cols(tf, m->transF[lv]);
        m->transIn_v[lv] = basis_rows(ti, m->transIn[lv]);
    }
    {
        std::vector<RowSrc> cs;
        for (int i = 0; i < nops; ++i) {
            const Op &op = *ops[i];
            const RowPanels &P = m->trans ? op.cpl_R : op.cpl;
            const void *v = m->trans ? op.cpl_R_vals.p : op.cpl_vals.p;
            cs.push_back({&P, 0, P.ngroups(), v, yho[i], xho[i]});
        }
        if (m->dt == H2B_F64)
            m->cpl_v = merge_rows<double>(cs, m->cpl, st);
        else if (m->dt == H2B_F32)
            m->cpl_v = merge_rows<float>(cs, m->cpl, st);
        else
            m->cpl_v = merge_rows<bf16_t>(cs, m->cpl, st);
    }
    m->transOut.resize(ndown);
    m->transOutT.resize(ndown);
    m->transOut_v.resize(ndown);
    m->transOutT_v.resize(ndown);
    for (size_t lv = 0; lv < ndown; ++lv) {
        std::vector<RowSrc> tr;
        std::vector<ColSrc> tt;
        for (int i = 0; i < nops; ++i) {
            const Basis &Bout = m->trans ? *ops[i]->colb : *ops[i]->rowb;
            const size_t n = Bout.fw_steps.size();
            if (lv >= n) continue;
            const auto &s = Bout.fw_steps[n - 1 - lv];
            tr.push_back({&Bout.trans, s.first, s.second, Bout.trans_vals.p, yho[i], yho[i]});
            const auto &b = Bout.bw_steps[lv];
            tt.push_back({&Bout.trans_T, b.first, b.second, Bout.trans_vals.p, yho[i], yho[i]});
        }
        m->transOut_v[lv] = basis_rows(tr, m->transOut[lv]);
        m->transOutT_v[lv] = basis_cols(tt, m->transOutT[lv]);
    }
    {
        std::vector<RowSrc> lo;
        std::vector<ColSrc> lt;
        std::vector<RowSrc> nr;
        for (int i = 0; i < nops; ++i) {
            const Op &op = *ops[i];
            const Basis &Bout = m->trans ? *op.colb : *op.rowb;
            lo.push_back({&Bout.leaf, 0, Bout.leaf.ngroups(), Bout.leaf_vals.p, yho[i], yo[i]});
            lt.push_back({&Bout.leaf_T, 0, Bout.leaf_T.ngroups(), Bout.leaf_vals.p, yo[i], yho[i]});
            const RowPanels &N = m->trans ? op.near_R : op.near;
            nr.push_back({&N, 0, N.ngroups(), m->trans ? op.near_R_vals.p : op.near_vals.p, yo[i], xo[i]});
        }
        m->leafOut_v = basis_rows(lo, m->leafOut);
        m->leafOutT_v = basis_cols(lt, m->leafOutT);
        m->near_v = merge_rows<double>(nr, m->near, st);
    }
    return m;
}

namespace {

template <typename F, typename C>
void merged_far(MergedBatch &m, hipStream_t st)
{
    const int rb = m.rb;
    F *xhat = m.xhat.as<F>(), *yhat = m.yhat.as<F>();
    double *xp = m.xp.as<double>(), *yp = m.yp.as<double>();
    if (rb == 1) {
        launch_colpanel<F, double, F>(m.leafF, 0, m.leafF.ngroups(), static_cast<const F *>(m.leafF_v), xp, xhat, st,
                                      Role::Leaf, false);
        for (size_t lv = 0; lv < m.transF.size(); ++lv)
            launch_colpanel<F, F, F>(m.transF[lv], 0, m.transF[lv].ngroups(), static_cast<const F *>(m.transF_v[lv]),
                                     xhat, xhat, st, Role::Transfer, false);
        launch_rowpanel<C, F, F>(m.cpl, 0, m.cpl.ngroups(), static_cast<const C *>(m.cpl_v), xhat, yhat, true, st,
                                 Role::Coupling);
        for (size_t lv = 0; lv < m.transOut.size(); ++lv)
            launch_rowpanelT<F, F, F>(m.transOut[lv], 0, m.transOut[lv].ngroups(),
                                      static_cast<const F *>(m.transOut_v[lv]), yhat, yhat, st, Role::Transfer);
        launch_rowpanelT<F, F, double>(m.leafOut, 0, m.leafOut.ngroups(), static_cast<const F *>(m.leafOut_v), yhat,
                                       yp, st, Role::Leaf);
        return;
    }
    bool leaf_done = false;
    if constexpr (std::is_same<F, double>::value) {
        if (m.leafIn.max_nrows <= 64) {
            launch_panel_mfma<double>(m.leafIn, 0, m.leafIn.ngroups(), rb, static_cast<const double *>(m.leafIn_v), xp,
                                      xhat, false, st);
            leaf_done = true;
        }
    }
    if (!leaf_done)
        launch_colpanel_mrhs<F, double, F>(m.leafF, 0, m.leafF.ngroups(), rb, static_cast<const F *>(m.leafF_v), xp,
                                           xhat, false, st, Role::Leaf);
    for (size_t lv = 0; lv < m.transF.size(); ++lv) {
        if (m.transIn[lv].max_nrows <= 64)
            launch_panel_mfma<F>(m.transIn[lv], 0, m.transIn[lv].ngroups(), rb,
                                 static_cast<const F *>(m.transIn_v[lv]), xhat, xhat, false, st);
        else
            launch_colpanel_mrhs<F, F, F>(m.transF[lv], 0, m.transF[lv].ngroups(), rb,
                                          static_cast<const F *>(m.transF_v[lv]), xhat, xhat, false, st,
                                          Role::Transfer);
    }
    const C *cv = static_cast<const C *>(m.cpl_v);
    bool cpl_done = false;
    if constexpr (std::is_same<F, C>::value) {
        if (m.cpl.max_nrows <= 64) {
            launch_panel_mfma<F>(m.cpl, 0, m.cpl.ngroups(), rb, cv, xhat, yhat, true, st);
            cpl_done = true;
        }
    }
    if (!cpl_done) {
        if constexpr (std::is_same<F, float>::value)
            launch_rowpanel_mrhs_mfma<C>(m.cpl, 0, m.cpl.ngroups(), rb, 32, cv, xhat, yhat, true, st);
        else
            launch_rowpanel_mrhs<C, F, F>(m.cpl, 0, m.cpl.ngroups(), rb, cv, xhat, yhat, true, st, Role::Coupling);
    }
    for (size_t lv = 0; lv < m.transOutT.size(); ++lv)
        launch_colpanel_mrhs<F, F, F>(m.transOutT[lv], 0, m.transOutT[lv].ngroups(), rb,
                                      static_cast<const F *>(m.transOutT_v[lv]), yhat, yhat, true, st,
                                      Role::Transfer);
    launch_colpanel_mrhs<F, F, double>(m.leafOutT, 0, m.leafOutT.ngroups(), rb, static_cast<const F *>(m.leafOutT_v),
                                       yhat, yp, true, st, Role::Leaf);
}

void merged_near(MergedBatch &m, hipStream_t st)
{
    double *xp = m.xp.as<double>(), *ypn = m.ypn.as<double>();
    if (m.rb == 1)
        launch_rowpanel<double, double, double>(m.near, 0, m.near.ngroups(), m.near_v, xp, ypn, true, st, Role::Near);
    else if (m.near.max_nrows <= 64)
        launch_panel_mfma<double>(m.near, 0, m.near.ngroups(), m.rb, m.near_v, xp, ypn, true, st);
    else
        launch_rowpanel_mrhs<double, double, double>(m.near, 0, m.near.ngroups(), m.rb, m.near_v, xp, ypn, true, st,
                                                     Role::Near);
}

template <typename F, typename C> void merged_run_t(MergedBatch &m, hipStream_t st)
{
    launch_fill_zero<F>(m.yhat.as<F>(), m.hout * m.rb, st);
    launch_fill_zero<double>(m.yp.as<double>(), m.nout * m.rb, st);
    launch_fill_zero<double>(m.ypn.as<double>(), m.nout * m.rb, st);
    if (m.nin > 0) {
        hipLaunchKernelGGL(k_gather_abs, dim3(grid_of(m.nin * m.rb)), dim3(BT), 0, st, m.gsrc.as<int64_t>(),
                           m.gld.as<int64_t>(), m.nin, m.nb, m.rb, m.xbase, m.xp.as<double>());
        hip_check(hipGetLastError(), "batch gather launch");
    }
    // the nearfield and the far field read only xp and write disjoint
    // vectors: two branches of the captured graph
    const std::vector<hipGraphNode_t> prep = capture_tail(st);
    merged_near(m, st);
    std::vector<hipGraphNode_t> ends = capture_tail(st);
    set_capture_tail(st, prep);
    merged_far<F, C>(m, st);
    const std::vector<hipGraphNode_t> far = capture_tail(st);
    ends.insert(ends.end(), far.begin(), far.end());
    set_capture_tail(st, ends);
    if (m.nout > 0) {
        hipLaunchKernelGGL(k_scatter_abs, dim3(grid_of(m.nout * m.nb)), dim3(BT), 0, st, m.sdst.as<int64_t>(),
                           m.sld.as<int64_t>(), m.salpha.as<double>(), m.nout, m.nb, m.rb, m.yp.as<double>(),
                           m.ypn.as<double>(), m.ybase);
        hip_check(hipGetLastError(), "batch scatter launch");
    }
}

}  // namespace

void merged_capture(MergedBatch &m, hipStream_t st)
{
    switch (m.dt) {
    case H2B_F64: merged_run_t<double, double>(m, st); break;
    case H2B_F32: merged_run_t<float, float>(m, st); break;
    default: merged_run_t<float, bf16_t>(m, st); break;
    }
}

int64_t merged_launches(const MergedBatch &m) { return (int64_t)(m.transF.size() + m.transOut.size()) + 9; }

}  // namespace h2b
