// Assembly of an H^2 operator (G or K) and the matrix-vector product driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

#include "device.hpp"
#include "linalg.hpp"
#include "op.hpp"

namespace h2b {

// ------------------------------------------------------------- panels

void transpose_panels(const RowPanels &rp, int g0, int g1, ColPanels &cp)
{
    // output group per distinct input segment (keyed by its start), blocks in
    // order of appearance
    std::map<int, std::vector<int>> by_out;  // seg_in -> list of (group, segment)
    std::map<int, int> out_len, out_tag;
    std::vector<std::pair<int, int>> refs;
    for (int g = g0; g < g1; ++g)
        for (int s = rp.seg_ptr[g]; s < rp.seg_ptr[g + 1]; ++s) {
            if (rp.seg_len[s] == 0 || rp.nrows[g] == 0) continue;  // contributes nothing
            by_out[rp.seg_in[s]].push_back((int)refs.size());
            out_len[rp.seg_in[s]] = rp.seg_len[s];
            out_tag[rp.seg_in[s]] = rp.seg_tag[s];
            refs.push_back({g, s});
        }
    // column offset of every segment inside its panel
    std::vector<int> c0(rp.seg_in.size(), 0);
    for (int g = g0; g < g1; ++g) {
        int c = 0;
        for (int s = rp.seg_ptr[g]; s < rp.seg_ptr[g + 1]; ++s) {
            c0[s] = c;
            c += rp.seg_len[s];
        }
    }
    for (auto &kv : by_out) {
        cp.out_begin.push_back(kv.first);
        cp.out_len.push_back(out_len[kv.first]);
        cp.out_tag.push_back(out_tag[kv.first]);
        cp.max_out = std::max(cp.max_out, out_len[kv.first]);
        for (int ref : kv.second) {
            int g = refs[ref].first, s = refs[ref].second;
            cp.b_val_off.push_back(rp.val_off[g]);
            cp.b_stride.push_back(rp.ncols[g]);
            cp.b_c0.push_back(c0[s]);
            cp.b_nrows.push_back(rp.nrows[g]);
            cp.b_in.push_back(rp.out_begin[g]);
            cp.b_tag.push_back(rp.group_tag[g]);
        }
        cp.blk_ptr.push_back((int32_t)cp.b_in.size());
    }
}

void regroup_transposed(const ColPanels &cp, RowPanels &out)
{
    out = RowPanels();
    for (int g = 0; g < cp.ngroups(); ++g) {
        out.begin_group(cp.out_tag[g], cp.out_begin[g], cp.out_len[g]);
        for (int b = cp.blk_ptr[g]; b < cp.blk_ptr[g + 1]; ++b) out.add_segment(cp.b_in[b], cp.b_nrows[b], cp.b_tag[b]);
        out.end_group();
    }
}

// -------------------------------------------------------------- bases

static int basis_quad_order(int m) { return (3 * m) / 2 + 1; }

QuadDev make_quad(int q)
{
    if (q < 1 || q > QMAX) fail(H2B_EINVAL, "quadrature order out of range");
    QuadDev Q{};
    std::vector<double> t, w;
    gauss_legendre_unit(q, t, w);
    Q.q = q;
    for (int i = 0; i < q; ++i) {
        Q.t[i] = t[i];
        Q.w[i] = w[i];
    }
    return Q;
}

// Column panels of the forward products over transposed panel copies: one
// output group per row-panel group, one block per segment (P^T rows of that
// segment, row stride = the group's row count).
static void forward_panels(const RowPanels &rp, ColPanels &cp)
{
    for (int g = 0; g < rp.ngroups(); ++g) {
        cp.out_begin.push_back(rp.out_begin[g]);
        cp.out_len.push_back(rp.nrows[g]);
        cp.max_out = std::max(cp.max_out, rp.nrows[g]);
        int c0 = 0;
        for (int s = rp.seg_ptr[g]; s < rp.seg_ptr[g + 1]; ++s) {
            cp.b_val_off.push_back(rp.val_off[g] + (int64_t)c0 * rp.nrows[g]);
            cp.b_stride.push_back(rp.nrows[g]);
            cp.b_c0.push_back(0);
            cp.b_nrows.push_back(rp.seg_len[s]);
            cp.b_in.push_back(rp.seg_in[s]);
            c0 += rp.seg_len[s];
        }
        cp.blk_ptr.push_back((int32_t)cp.b_in.size());
    }
}

// Structure of a cluster basis with the given rank per cluster.
void build_basis_structure(Basis &B, const std::vector<int> &ranks, hipStream_t st)
{
    const Tree &T = *B.tree;
    const int64_t nc = T.nclusters();
    B.rank = ranks;
    B.hat_off.resize(nc + 1);
    B.hat_off[0] = 0;
    for (int64_t c = 0; c < nc; ++c) B.hat_off[c + 1] = B.hat_off[c] + B.rank[c];
    B.hat_total = B.hat_off[nc];
    if (B.hat_total > INT32_MAX) fail(H2B_ENOTSUP, "too many cluster coefficients for 32-bit offsets");
    // leaves: V_t^T, k x |t|
    for (int c : T.leaves) {
        B.leaf.begin_group(c, (int)B.hat_off[c], B.rank[c]);
        B.leaf.add_segment(T.begin[c], T.size(c), c);
        B.leaf.end_group();
    }
    transpose_panels(B.leaf, 0, B.leaf.ngroups(), B.leaf_T);
    // transfers, deepest parents first
    B.fw_steps.clear();
    for (int lev = T.nlevels - 2; lev >= 0; --lev) {
        int g0 = B.trans.ngroups();
        for (int c : T.by_level[lev]) {
            if (T.nchild[c] == 0) continue;
            B.trans.begin_group(c, (int)B.hat_off[c], B.rank[c]);
            for (int ch : {T.child0[c], T.child1[c]})
                B.trans.add_segment((int)B.hat_off[ch], B.rank[ch], ch);
            B.trans.end_group();
        }
        B.fw_steps.push_back({g0, B.trans.ngroups()});
    }
    // backward: top level first; transposed panels of each step
    B.bw_steps.clear();
    for (auto it = B.fw_steps.rbegin(); it != B.fw_steps.rend(); ++it) {
        int o0 = B.trans_T.ngroups();
        transpose_panels(B.trans, it->first, it->second, B.trans_T);
        B.bw_steps.push_back({o0, B.trans_T.ngroups()});
    }
    forward_panels(B.leaf, B.leaf_F);
    forward_panels(B.trans, B.trans_F);
    B.leaf_F.upload(st);
    B.trans_F.upload(st);
    build_level_descriptors(B, st);
}

void transpose_basis_values(Basis &B, h2b_dtype dt, hipStream_t st)
{
    const size_t esz = (dt == H2B_F64) ? sizeof(double) : sizeof(float);
    B.leafT_vals.alloc(esz * std::max<int64_t>(B.leaf.total, 1));
    B.transT_vals.alloc(esz * std::max<int64_t>(B.trans.total, 1));
    if (dt == H2B_F64) {
        launch_transpose_panels<double>(B.leaf, B.leaf_vals.as<double>(), B.leafT_vals.as<double>(), st);
        launch_transpose_panels<double>(B.trans, B.trans_vals.as<double>(), B.transT_vals.as<double>(), st);
    } else {
        launch_transpose_panels<float>(B.leaf, B.leaf_vals.as<float>(), B.leafT_vals.as<float>(), st);
        launch_transpose_panels<float>(B.trans, B.trans_vals.as<float>(), B.transT_vals.as<float>(), st);
    }
    hip_check(hipStreamSynchronize(st), "basis transpose");
}


template <typename T>
static void assemble_basis(Basis &B, int m, const DevMem &axes, const GeoDev &geo, hipStream_t st)
{
    B.leaf_vals.alloc(sizeof(T) * std::max<int64_t>(B.leaf.total, 1));
    B.trans_vals.alloc(sizeof(T) * std::max<int64_t>(B.trans.total, 1));
    QuadDev Q = make_quad(basis_quad_order(m));
    launch_leaf_basis<T>(B.dlp_cols, B.leaf, B.perm_dev, axes.as<double>(), m, geo, Q,
                         B.leaf_vals.as<T>(), st);
    launch_transfer<T>(B.trans, axes.as<double>(), m, B.trans_vals.as<T>(), st);
}

// ---------------------------------------------------------- operator

// Nearfield entries of G, or of K with every triangle pair integrated once
// per row: the sorted triangles around each group's column vertices go to
// the device for the assembly and are freed afterwards.
static void assemble_near(Op &op, const QuadDev &Qn, hipStream_t st)
{
    if (op.kernel == H2B_SLP) {
        launch_near_assemble(H2B_SLP, op.near, op.rowb->perm_dev, op.colb->perm_dev, op.geo, Qn,
                             op.near_vals.as<double>(), st);
        return;
    }
    const Tree &C = *op.colb->tree;
    const Mesh &M = *C.mesh;
    const RowPanels &N = op.near;
    const int ng = N.ngroups();
    std::vector<std::vector<int32_t>> per(ng);
    parallel_for(ng, [&](int64_t g) {
        std::vector<int32_t> &v = per[g];
        for (int s = N.seg_ptr[g]; s < N.seg_ptr[g + 1]; ++s)
            for (int p = N.seg_in[s]; p < N.seg_in[s] + N.seg_len[s]; ++p) {
                const int j = C.perm[p];
                for (int64_t a = M.vt_ptr[j]; a < M.vt_ptr[j + 1]; ++a) v.push_back(M.vt_idx[a]);
            }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    });
    std::vector<int64_t> lptr(ng + 1, 0);
    for (int g = 0; g < ng; ++g) lptr[g + 1] = lptr[g] + (int64_t)per[g].size();
    std::vector<int32_t> lst(std::max<int64_t>(lptr[ng], 1));
    parallel_for(ng, [&](int64_t g) { std::copy(per[g].begin(), per[g].end(), lst.begin() + lptr[g]); });
    per.clear();
    DevMem dptr, dlst;
    dptr.alloc(sizeof(int64_t) * lptr.size());
    dlst.alloc(sizeof(int32_t) * lst.size());
    hip_check(hipMemcpyAsync(dptr.p, lptr.data(), sizeof(int64_t) * lptr.size(), hipMemcpyHostToDevice, st),
              "triangle list upload");
    hip_check(hipMemcpyAsync(dlst.p, lst.data(), sizeof(int32_t) * lst.size(), hipMemcpyHostToDevice, st),
              "triangle list upload");
    launch_near_assemble_dlp(N, dptr.as<int64_t>(), dlst.as<int32_t>(), op.rowb->perm_dev, op.colb->perm_dev,
                             op.geo, Qn, op.near_vals.as<double>(), st);
    hip_check(hipStreamSynchronize(st), "double-layer nearfield assembly");
}

Op::~Op()
{
    for (auto &set : ev)
        for (auto &e : set)
            if (e) (void)hipEventDestroy(e);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
}

static void upload_tree(Basis &B, hipStream_t st)
{
    Packer pk;
    pk.add(B.tree->perm, const_cast<int32_t **>(&B.perm_dev));
    pk.upload(B.perm_mem, st);
}

static void upload_axes(const Tree &T, int m, DevMem &mem, hipStream_t st)
{
    std::vector<double> ax((size_t)T.nclusters() * 3 * m);
    for (int64_t c = 0; c < T.nclusters(); ++c) cheb_axes(T, (int)c, m, &ax[(size_t)c * 3 * m]);
    mem.alloc(ax.size() * sizeof(double));
    hip_check(hipMemcpyAsync(mem.p, ax.data(), ax.size() * sizeof(double), hipMemcpyHostToDevice, st),
              "axes upload");
    hip_check(hipStreamSynchronize(st), "axes upload");
}

std::unique_ptr<Op> assemble_op(std::shared_ptr<const Blocks> blocks, h2b_kernel kernel,
                                const h2b_params &p, hipStream_t st)
{
    if (p.order_m < 1 || p.order_m > MMAX) fail(H2B_EINVAL, "order_m must be in 1..6");
    if (p.q_near < 2 || p.q_near > QMAX) fail(H2B_EINVAL, "q_near must be in 2..16");
    if (p.farfield_dtype != H2B_F64 && p.farfield_dtype != H2B_F32 && p.farfield_dtype != H2B_BF16)
        fail(H2B_EINVAL, "farfield_dtype must be H2B_F64, H2B_F32 or H2B_BF16");
    if (!(p.recompress_tol >= 0.0)) fail(H2B_EINVAL, "recompress_tol must be >= 0");
    if (kernel == H2B_SLP && blocks->cols->space != H2B_P0)
        fail(H2B_EINVAL, "the single-layer matrix needs a P0 column tree");
    if (kernel == H2B_DLP && blocks->cols->space != H2B_P1)
        fail(H2B_EINVAL, "the double-layer matrix needs a P1 column tree");
    if (kernel != H2B_SLP && kernel != H2B_DLP) fail(H2B_EINVAL, "unknown kernel");
    // ranks above 64 (orders 5-6, cross-approximation bases) are recompressed
    // in FP64 only
    if (p.recompress_tol > 0.0 && p.order_m > 4 && p.farfield_dtype != H2B_F64)
        fail(H2B_ENOTSUP, "an FP32 or BF16 far field with recompression supports order_m <= 4");
    if (!(p.gca_tol >= 0.0) || !std::isfinite(p.gca_tol)) fail(H2B_EINVAL, "gca_tol must be finite and >= 0");
    const bool gca = p.gca_tol > 0.0;
    if (gca && p.recompress_tol > 0.0 && p.farfield_dtype != H2B_F64)
        fail(H2B_ENOTSUP, "the Green cross approximation is recompressed in FP64 only");
    if (kernel == H2B_SLP && blocks->rows != blocks->cols)
        fail(H2B_EINVAL, "the single-layer matrix needs one cluster tree for its rows and columns");
    // Reduced-precision storage keeps the error of the far field at the level
    // of the FP32/BF16 rounding only for orthonormal cluster bases, i.e. after
    // the algebraic recompression; interpolation and cross-approximation bases
    // are not orthonormal and amplify it.
    if (p.farfield_dtype != H2B_F64 && !(p.recompress_tol > 0.0))
        fail(H2B_ENOTSUP, "an FP32 or BF16 far field needs orthonormal bases (recompress_tol > 0)");
    if (p.recompute_coupling && (p.farfield_dtype != H2B_F64 || gca))
        fail(H2B_ENOTSUP, "evaluated couplings need an FP64 interpolation far field (no gca_tol)");

    auto op = std::make_unique<Op>();
    op->blocks = blocks;
    op->kernel = kernel;
    op->params = p;
    op->recompute = p.recompute_coupling != 0;
    const Tree &R = *blocks->rows, &C = *blocks->cols;
    const Mesh &M = *R.mesh;
    op->nrows = R.n;
    op->ncols = C.n;
    const int m = p.order_m;
    const int k = m * m * m;

    // geometry
    {
        Packer pk;
        pk.add(M.vx, const_cast<double **>(&op->geo.vx));
        pk.add(M.vy, const_cast<double **>(&op->geo.vy));
        pk.add(M.vz, const_cast<double **>(&op->geo.vz));
        pk.add(M.t0, const_cast<int32_t **>(&op->geo.t0));
        pk.add(M.t1, const_cast<int32_t **>(&op->geo.t1));
        pk.add(M.t2, const_cast<int32_t **>(&op->geo.t2));
        pk.add(M.nx, const_cast<double **>(&op->geo.nx));
        pk.add(M.ny, const_cast<double **>(&op->geo.ny));
        pk.add(M.nz, const_cast<double **>(&op->geo.nz));
        pk.add(M.vt_ptr, const_cast<int64_t **>(&op->geo.vt_ptr));
        pk.add(M.vt_idx, const_cast<int32_t **>(&op->geo.vt_idx));
        pk.upload(op->geo_mem, st);
    }

    // bases
    op->rowb = std::make_shared<Basis>();
    op->rowb->tree = blocks->rows;
    op->rowb->dlp_cols = false;
    upload_tree(*op->rowb, st);
    if (kernel == H2B_SLP) {
        op->colb = op->rowb;
    } else {
        op->colb = std::make_shared<Basis>();
        op->colb->tree = blocks->cols;
        op->colb->dlp_cols = true;
        upload_tree(*op->colb, st);
    }
    upload_axes(R, m, op->rowb->axes, st);
    if (op->colb != op->rowb) upload_axes(C, m, op->colb->axes, st);
    std::vector<Basis *> bases{op->rowb.get()};
    if (op->colb != op->rowb) bases.push_back(op->colb.get());
    // Green cross approximation: pivots and nested bases first (host), their
    // ranks shape the basis and coupling panels
    GcaBases gb, gbc;
    if (gca) {
        gb = gca_bases(R, m, p.gca_tol);
        if (op->colb != op->rowb) gbc = gca_bases(C, m, p.gca_tol);
    }
    for (Basis *B : bases) {
        const std::vector<int> &gr = B == op->rowb.get() ? gb.rank : gbc.rank;
        build_basis_structure(*B, gca ? gr : std::vector<int>(B->tree->nclusters(), k), st);
        B->leaf.upload(st);
        B->leaf_T.upload(st);
        B->trans.upload(st);
        B->trans_T.upload(st);
    }

    // nearfield panels (rows grouped by row leaf, blocks in construction order)
    {
        std::vector<std::vector<int>> per_row(R.nclusters());
        for (size_t b = 0; b < blocks->near_t.size(); ++b) per_row[blocks->near_t[b]].push_back((int)b);
        for (int t : R.leaves) {
            if (per_row[t].empty()) continue;
            op->near.begin_group(t, R.begin[t], R.size(t));
            for (int b : per_row[t]) {
                int s = blocks->near_s[b];
                op->near.add_segment(C.begin[s], C.size(s), s);
            }
            op->near.end_group();
        }
        transpose_panels(op->near, 0, op->near.ngroups(), op->near_T);
        op->near.upload(st);
        op->near_T.upload(st);
    }
    // coupling panels (grouped by row cluster)
    {
        std::vector<std::vector<int>> per_row(R.nclusters());
        for (size_t b = 0; b < blocks->far_t.size(); ++b) per_row[blocks->far_t[b]].push_back((int)b);
        for (int64_t t = 0; t < R.nclusters(); ++t) {
            if (per_row[t].empty()) continue;
            op->cpl.begin_group((int)t, (int)op->rowb->hat_off[t], op->rowb->rank[t]);
            for (int b : per_row[t]) {
                int s = blocks->far_s[b];
                op->cpl.add_segment((int)op->colb->hat_off[s], op->colb->rank[s], s);
            }
            op->cpl.end_group();
        }
        transpose_panels(op->cpl, 0, op->cpl.ngroups(), op->cpl_T);
        op->cpl.upload(st);
        op->cpl_T.upload(st);
    }

    // values
    op->near_vals.alloc(sizeof(double) * std::max<int64_t>(op->near.total, 1));
    QuadDev Qn = make_quad(p.q_near);
    assemble_near(*op, Qn, st);
    // with recompression the interpolation operator is built in FP64 first
    const bool rc = p.recompress_tol > 0.0;
    const h2b_dtype adt = rc ? H2B_F64 : p.farfield_dtype;
    if (gca) {
        set_gca_values(*op, gb, op->colb != op->rowb ? gbc : gb, st);
    } else {
    // evaluated couplings are not stored, except transiently for the recompression
    const bool store_cpl = !op->recompute || rc;
    if (store_cpl) op->cpl_vals.alloc(coupling_size(adt) * std::max<int64_t>(op->cpl.total, 1));
    for (Basis *B : bases) {
        if (adt == H2B_F64)
            assemble_basis<double>(*B, m, B->axes, op->geo, st);
        else
            assemble_basis<float>(*B, m, B->axes, op->geo, st);
        transpose_basis_values(*B, adt, st);
    }
    const double *rax = op->rowb->axes.as<double>(), *cax = op->colb->axes.as<double>();
    if (!store_cpl)
        ;
    else if (adt == H2B_F64)
        launch_coupling<double>(op->cpl, rax, cax, m, op->cpl_vals.as<double>(), st);
    else if (adt == H2B_F32)
        launch_coupling<float>(op->cpl, rax, cax, m, op->cpl_vals.as<float>(), st);
    else
        launch_coupling<bf16_t>(op->cpl, rax, cax, m, op->cpl_vals.as<bf16_t>(), st);
    }
    hip_check(hipStreamSynchronize(st), "assembly");
    if (rc) recompress_op(*op, p.recompress_tol, st);
    if (p.transposed_copy) make_transposed_copies(*op, st);
    if (op->recompute) setup_recompute(*op, st);
    // the once-per-pair kernel keeps a leaf's rows in LDS: leaves of at most 64
    if (p.symmetric_near && kernel == H2B_SLP && blocks->rows == blocks->cols && op->near.max_nrows <= 64 &&
        op->near.ngroups() > 0)
        make_symmetric_near(*op, st);
    // the far field of G once per pair: stored FP64 or FP32 couplings, kernel
    // values at interpolation points or quadrature entries of well-separated
    // pivot triangles (both symmetric to rounding)
    if (op->sym && !op->recompute && p.farfield_dtype != H2B_BF16 && op->rowb == op->colb &&
        op->cpl.max_nrows <= SYMCPL_MAX_RANK && op->cpl.ngroups() > 0)
        make_symmetric_coupling(*op, st);

    // work vectors
    const size_t wsz = basis_size(p.farfield_dtype);
    const int64_t nmax = std::max(op->nrows, op->ncols);
    const int64_t hmax = std::max(op->rowb->hat_total, op->colb->hat_total);
    op->xp.alloc(sizeof(double) * nmax);
    op->yp.alloc(sizeof(double) * nmax);
    op->ypn.alloc(sizeof(double) * nmax);
    hip_check(hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking), "stream create");
    hip_check(hipEventCreateWithFlags(&op->fork, hipEventDisableTiming), "event create");
    hip_check(hipEventCreateWithFlags(&op->join, hipEventDisableTiming), "event create");
    op->xhat.alloc(wsz * std::max<int64_t>(hmax, 1));
    op->yhat.alloc(wsz * std::max<int64_t>(hmax, 1));
    if (op->rowb->has_proj) {
        const int64_t kc = (int64_t)k * std::max(R.nclusters(), C.nclusters());
        op->xt.alloc(sizeof(double) * kc);
        op->yt.alloc(sizeof(double) * kc);
    }
    return op;
}

void make_transposed_copies(Op &op, hipStream_t st)
{
    const h2b_dtype dt = op.params.farfield_dtype;
    if (!op.has_R) {
        regroup_transposed(op.near_T, op.near_R);
        regroup_transposed(op.cpl_T, op.cpl_R);
        op.near_R.upload(st);
        op.cpl_R.upload(st);
        op.near_R_vals.alloc(sizeof(double) * std::max<int64_t>(op.near_R.total, 1));
        if (!op.recompute) op.cpl_R_vals.alloc(coupling_size(dt) * std::max<int64_t>(op.cpl_R.total, 1));
    }
    launch_regroup_transpose<double>(op.near_T, op.near_R, op.near_vals.as<double>(), op.near_R_vals.as<double>(),
                                     st);
    if (op.recompute)
        ;  // no stored couplings: cpl_R only groups the blocks by column cluster
    else if (dt == H2B_F64)
        launch_regroup_transpose<double>(op.cpl_T, op.cpl_R, op.cpl_vals.as<double>(),
                                         op.cpl_R_vals.as<double>(), st);
    else if (dt == H2B_F32)
        launch_regroup_transpose<float>(op.cpl_T, op.cpl_R, op.cpl_vals.as<float>(), op.cpl_R_vals.as<float>(),
                                        st);
    else
        launch_regroup_transpose<bf16_t>(op.cpl_T, op.cpl_R, op.cpl_vals.as<bf16_t>(),
                                         op.cpl_R_vals.as<bf16_t>(), st);
    hip_check(hipStreamSynchronize(st), "transposed copies");
    op.has_R = true;
}

// --------------------------------------------------------------- product
//
// F: type of the bases and of the cluster coefficients (double for F64, float
// otherwise); C: storage type of the coupling matrices (double, float, bf16).

template <typename F>
static void forward(const Basis &B, const double *xp, F *xhat, hipStream_t st)
{
    if (B.lev) {
        forward_levels<F>(B, xp, xhat, st);
        return;
    }
    launch_colpanel<F, double, F>(B.leaf_F, 0, B.leaf_F.ngroups(), B.leafT_vals.as<F>(), xp, xhat, st,
                                  Role::Leaf, false);
    for (auto &s : B.fw_steps)
        launch_colpanel<F, F, F>(B.trans_F, s.first, s.second, B.transT_vals.as<F>(), xhat, xhat, st,
                                 Role::Transfer, false);
}

template <typename F>
static void backward(const Basis &B, F *yhat, double *yp, hipStream_t st)
{
    if (B.lev) {
        backward_levels<F>(B, yhat, yp, st);
        return;
    }
    for (auto it = B.fw_steps.rbegin(); it != B.fw_steps.rend(); ++it)
        launch_rowpanelT<F, F, F>(B.trans, it->first, it->second, B.trans_vals.as<F>(), yhat, yhat, st,
                                  Role::Transfer);
    launch_rowpanelT<F, F, double>(B.leaf, 0, B.leaf.ngroups(), B.leaf_vals.as<F>(), yhat, yp, st, Role::Leaf);
}

// Events: [0] start, [1] after gather, [2] after forward, [3] after coupling,
// [4] after backward (caller's stream); [5] nearfield start, [6] nearfield end
// (side stream); [7] after the join, [8] after scatter (caller's stream).  The
// coupling phase brackets one kernel launch, the nearfield phase one (two for
// the once-per-pair storage of G: rows and column sums, then their reduction).
static hipEvent_t *event_set(Op &op, hipStream_t st)
{
    if (!op.timing) return nullptr;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return nullptr;
    if (op.nev == op.ev.size()) {
        std::array<hipEvent_t, 9> set{};
        for (auto &e : set) hip_check(hipEventCreate(&e), "event create");
        op.ev.push_back(set);
    }
    return op.ev[op.nev++].data();
}

// Stream of the nearfield: the operator's side stream, which waits for
// everything queued on st so far (fork), or st itself when overlap is off or
// while st is being captured into a graph (no capture spans two streams: a
// captured product forms its branches on the captured stream).
static hipStream_t fork_side(Op &op, hipStream_t st)
{
    if (!op.overlap) return st;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cs), "capture status");
    if (cs != hipStreamCaptureStatusNone) return st;
    hip_check(hipEventRecord(op.fork, st), "event record");
    hip_check(hipStreamWaitEvent(op.side, op.fork, 0), "stream wait");
    return op.side;
}

// st waits for everything queued on the nearfield stream ns so far (join).
static void join_side(Op &op, hipStream_t ns, hipStream_t st)
{
    if (ns == st) return;
    hip_check(hipEventRecord(op.join, ns), "event record");
    hip_check(hipStreamWaitEvent(st, op.join, 0), "stream wait");
}

// Work vectors of one product (rb = 1 for a single vector, else the block
// width): the operator's own, or views into the static scratch array of the
// allocation-free entry point.  `sym` allows the once-per-pair nearfield of G
// (whose column sums live in the operator); `timed` allows phase events.
struct Work {
    double *xp, *yp, *ypn;
    void *xhat, *yhat;
    bool sym, timed;
    double *xt, *yt;  // interpolation coefficients of evaluated couplings on recompressed bases
};

// The four pieces of one product.  Prepare clears the outputs and gathers x
// into cluster order; Near (nearfield into ypn) and Far (forward
// transformation, coupling, backward transformation into yp) both read only
// xp and write disjoint buffers, so they may run concurrently; Finish adds
// alpha (yp + ypn) to y in the caller's order.  `mark` records the phase
// events of a timed product (NULL when untimed).
enum class Piece { Prepare, Near, Far, Finish };

template <typename F, typename C>
static void product_piece(Op &op, const Work &w, int trans, double alpha, const double *x, double *y, Piece pc,
                          hipStream_t st, hipEvent_t *ev)
{
    const Basis &Bin = trans ? *op.rowb : *op.colb;
    const Basis &Bout = trans ? *op.colb : *op.rowb;
    const int64_t nin = trans ? op.nrows : op.ncols;
    const int64_t nout = trans ? op.ncols : op.nrows;
    double *xp = w.xp, *yp = w.yp, *ypn = w.ypn;
    F *xhat = static_cast<F *>(w.xhat), *yhat = static_cast<F *>(w.yhat);
    auto mark = [&](int i) {
        if (ev) hip_check(hipEventRecord(ev[i], st), "event record");
    };
    switch (pc) {
    case Piece::Prepare:
        // the nearfield's output is cleared here too: on its own stream the
        // fill would wait behind the forward transformation's workgroups
        launch_fill_zero<F>(yhat, Bout.hat_total, st);
        launch_fill_zero<double>(yp, nout, st);
        launch_fill_zero<double>(ypn, nout, st);
        mark(0);
        launch_gather(Bin.perm_dev, nin, 1, x, nin, xp, st);
        mark(1);
        break;
    case Piece::Near:
        mark(5);
        if (op.sym && w.sym)
            symmetric_near_product(op, trans, xp, ypn, st);
        else if (!trans)
            launch_rowpanel<double, double, double>(op.near, 0, op.near.ngroups(), op.near_vals.as<double>(), xp,
                                                    ypn, true, st, Role::Near);
        else if (op.has_R)
            launch_rowpanel<double, double, double>(op.near_R, 0, op.near_R.ngroups(),
                                                    op.near_R_vals.as<double>(), xp, ypn, true, st, Role::Near);
        else
            launch_colpanel<double, double, double>(op.near_T, 0, op.near_T.ngroups(), op.near_vals.as<double>(),
                                                    xp, ypn, st, Role::Near);
        mark(6);
        break;
    case Piece::Far:
        forward<F>(Bin, xp, xhat, st);
        mark(2);
        if constexpr (std::is_same<F, double>::value) {
            if (op.recompute) {
                recompute_coupling(op, trans, 1, xhat, yhat, w.xt, w.yt, st);
                mark(3);
                backward<F>(Bout, yhat, yp, st);
                mark(4);
                break;
            }
        }
        if constexpr (std::is_same<F, C>::value) {
            if (op.symcpl && w.sym) {
                symmetric_coupling_product(op, xhat, yhat, st);
                mark(3);
                backward<F>(Bout, yhat, yp, st);
                mark(4);
                break;
            }
        }
        if (!trans)
            launch_rowpanel<C, F, F>(op.cpl, 0, op.cpl.ngroups(), op.cpl_vals.as<C>(), xhat, yhat, true, st,
                                     Role::Coupling);
        else if (op.has_R)
            launch_rowpanel<C, F, F>(op.cpl_R, 0, op.cpl_R.ngroups(), op.cpl_R_vals.as<C>(), xhat, yhat, true,
                                     st, Role::Coupling);
        else
            launch_colpanel<C, F, F>(op.cpl_T, 0, op.cpl_T.ngroups(), op.cpl_vals.as<C>(), xhat, yhat, st,
                                     Role::Coupling);
        mark(3);
        backward<F>(Bout, yhat, yp, st);
        mark(4);
        break;
    case Piece::Finish:
        launch_scatter_add(Bout.perm_dev, nout, 1, alpha, yp, ypn, y, nout, st);
        mark(8);
        break;
    }
}

std::vector<hipGraphNode_t> capture_tail(hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipGraphNode_t *d = nullptr;
    size_t nd = 0;
    hip_check(hipStreamGetCaptureInfo_v2(st, &cs, nullptr, nullptr, &d, &nd), "capture info");
    return std::vector<hipGraphNode_t>(d, d + nd);
}

void set_capture_tail(hipStream_t st, std::vector<hipGraphNode_t> deps)
{
    hip_check(hipStreamUpdateCaptureDependencies(st, deps.empty() ? nullptr : deps.data(), deps.size(),
                                                 hipStreamSetCaptureDependencies),
              "capture dependencies");
}

template <typename F, typename C>
static void product_one(Op &op, const Work &w, int trans, double alpha, const double *x, double *y, hipStream_t st)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hip_check(hipStreamIsCapturing(st, &cs), "capture status");
    if (cs != hipStreamCaptureStatusNone && op.overlap) {
        // captured into a graph: the nearfield and the far field become two
        // parallel branches after the gather, made on this one stream by
        // resetting what the next captured work depends on
        product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Prepare, st, nullptr);
        const std::vector<hipGraphNode_t> prep = capture_tail(st);
        product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Near, st, nullptr);
        std::vector<hipGraphNode_t> ends = capture_tail(st);
        set_capture_tail(st, prep);
        product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Far, st, nullptr);
        const std::vector<hipGraphNode_t> far = capture_tail(st);
        ends.insert(ends.end(), far.begin(), far.end());
        set_capture_tail(st, ends);
        product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Finish, st, nullptr);
        return;
    }
    hipEvent_t *ev = w.timed ? event_set(op, st) : nullptr;
    product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Prepare, st, ev);
    // nearfield on the side stream from here, or on st after the far field
    hipStream_t ns = fork_side(op, st);
    if (ns != st) product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Near, ns, ev);
    product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Far, st, ev);
    if (ns == st) product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Near, st, ev);
    join_side(op, ns, st);
    if (ev) hip_check(hipEventRecord(ev[7], st), "event record");
    product_piece<F, C>(op, w, trans, alpha, x, y, Piece::Finish, st, ev);
}

// ------------------------------------------------ many right-hand sides

// Block width for nrhs right-hand sides: the block kernels exist for 16, 32
// and 64 columns only.
static int block_width(const Op &op, int nrhs)
{
    if (op.tune_rb > 0) return op.tune_rb;
    return nrhs <= 16 ? 16 : nrhs <= 32 ? 32 : 64;
}

static void ensure_block_buffers(Op &op, int rb)
{
    if (rb != 16 && rb != 32 && rb != 64) fail(H2B_EINVAL, "block width must be 16, 32 or 64");
    if (op.mrhs_rb >= rb) return;
    const int64_t nmax = std::max(op.nrows, op.ncols);
    const int64_t hmax = std::max<int64_t>(std::max(op.rowb->hat_total, op.colb->hat_total), 1);
    const size_t fsz = basis_size(op.params.farfield_dtype);
    op.xpb.alloc(sizeof(double) * nmax * rb);
    op.ypb.alloc(sizeof(double) * nmax * rb);
    op.xhatb.alloc(fsz * hmax * rb);
    op.yhatb.alloc(fsz * hmax * rb);
    op.ypbn.alloc(sizeof(double) * nmax * rb);
    if (op.rowb->has_proj) {
        const int k = op.params.order_m * op.params.order_m * op.params.order_m;
        const int64_t kc = (int64_t)k * std::max(op.rowb->tree->nclusters(), op.colb->tree->nclusters());
        op.xtb.alloc(sizeof(double) * kc * rb);
        op.ytb.alloc(sizeof(double) * kc * rb);
    }
    op.mrhs_rb = rb;
}

template <typename F, typename C>
static void coupling_block(Op &op, int trans, int rb, int kc, const F *xhat, F *yhat, hipStream_t st,
                           double *xt = nullptr, double *yt = nullptr)
{
    if constexpr (std::is_same<F, double>::value) {
        if (op.recompute) {
            recompute_coupling(op, trans, rb, xhat, yhat, xt ? xt : op.xtb.as<double>(), yt ? yt : op.ytb.as<double>(),
                               st);
            return;
        }
    }
    if (trans && !op.has_R) {
        launch_colpanel_mrhs<C, F, F>(op.cpl_T, 0, op.cpl_T.ngroups(), rb, op.cpl_vals.as<C>(), xhat, yhat, true,
                                      st, Role::Coupling);
        return;
    }
    const RowPanels &P = trans ? op.cpl_R : op.cpl;
    const C *vals = trans ? op.cpl_R_vals.as<C>() : op.cpl_vals.as<C>();
    if constexpr (std::is_same<F, C>::value) {
        // FP32 or FP64: matrix cores, columns split over the waves
        if (P.max_nrows <= 64) {
            launch_panel_mfma<F>(P, 0, P.ngroups(), rb, vals, xhat, yhat, true, st);
            return;
        }
    }
    if constexpr (std::is_same<F, float>::value)
        launch_rowpanel_mrhs_mfma<C>(P, 0, P.ngroups(), rb, kc, vals, xhat, yhat, true, st);
    else
        launch_rowpanel_mrhs<C, F, F>(P, 0, P.ngroups(), rb, vals, xhat, yhat, true, st, Role::Coupling);
}

// Product for nb <= rb right-hand sides at once (block vectors row-major).
template <typename F, typename C>
static void product_block(Op &op, const Work &w, int trans, double alpha, const double *x, int64_t ldx, double *y,
                          int64_t ldy, int nb, int rb, hipStream_t st)
{
    const Basis &Bin = trans ? *op.rowb : *op.colb;
    const Basis &Bout = trans ? *op.colb : *op.rowb;
    const int64_t nin = trans ? op.nrows : op.ncols;
    const int64_t nout = trans ? op.ncols : op.nrows;
    double *xp = w.xp, *yp = w.yp, *ypn = w.ypn;
    F *xhat = static_cast<F *>(w.xhat), *yhat = static_cast<F *>(w.yhat);
    hipEvent_t *ev = w.timed ? event_set(op, st) : nullptr;
    auto mark = [&](int i, hipStream_t s) {
        if (ev) hip_check(hipEventRecord(ev[i], s), "event record");
    };
    launch_fill_zero<F>(yhat, Bout.hat_total * rb, st);
    launch_fill_zero<double>(yp, nout * rb, st);
    launch_fill_zero<double>(ypn, nout * rb, st);
    mark(0, st);
    launch_gather_mrhs(Bin.perm_dev, nin, nb, rb, x, ldx, xp, st);
    mark(1, st);
    hipStream_t ns = fork_side(op, st);
    auto nearfield = [&] {
        mark(5, ns);
        const RowPanels &NP = trans ? op.near_R : op.near;
        const double *nv = trans ? op.near_R_vals.as<double>() : op.near_vals.as<double>();
        if ((!trans || op.has_R) && NP.max_nrows <= 64)
            launch_panel_mfma<double>(NP, 0, NP.ngroups(), rb, nv, xp, ypn, true, ns);
        else if (!trans)
            launch_rowpanel_mrhs<double, double, double>(op.near, 0, op.near.ngroups(), rb,
                                                         op.near_vals.as<double>(), xp, ypn, true, ns, Role::Near);
        else if (op.has_R)
            launch_rowpanel_mrhs<double, double, double>(op.near_R, 0, op.near_R.ngroups(), rb,
                                                         op.near_R_vals.as<double>(), xp, ypn, true, ns, Role::Near);
        else
            launch_colpanel_mrhs<double, double, double>(op.near_T, 0, op.near_T.ngroups(), rb,
                                                         op.near_vals.as<double>(), xp, ypn, true, ns, Role::Near);
        mark(6, ns);
    };
    if (ns != st) nearfield();
    // forward transformation: row panels V_t^T and [E_c0^T | E_c1^T] on matrix
    // cores where types and sizes allow, else column products over the copies
    bool leaf_done = false;
    if constexpr (std::is_same<F, double>::value) {
        if (Bin.leaf.max_nrows <= 64) {
            launch_panel_mfma<double>(Bin.leaf, 0, Bin.leaf.ngroups(), rb, Bin.leaf_vals.as<double>(), xp, xhat,
                                      false, st);
            leaf_done = true;
        }
    }
    if (!leaf_done)
        launch_colpanel_mrhs<F, double, F>(Bin.leaf_F, 0, Bin.leaf_F.ngroups(), rb, Bin.leafT_vals.as<F>(), xp,
                                           xhat, false, st, Role::Leaf);
    for (auto &s : Bin.fw_steps) {
        if (Bin.trans.max_nrows <= 64)
            launch_panel_mfma<F>(Bin.trans, s.first, s.second, rb, Bin.trans_vals.as<F>(), xhat, xhat, false, st);
        else
            launch_colpanel_mrhs<F, F, F>(Bin.trans_F, s.first, s.second, rb, Bin.transT_vals.as<F>(), xhat, xhat,
                                          false, st, Role::Transfer);
    }
    mark(2, st);
    coupling_block<F, C>(op, trans, rb, op.tune_kc, xhat, yhat, st, w.xt, w.yt);
    mark(3, st);
    // backward transformation: column products over the panels (row panels of
    // single children were measured slower for these small matrices)
    for (auto &s : Bout.bw_steps)
        launch_colpanel_mrhs<F, F, F>(Bout.trans_T, s.first, s.second, rb, Bout.trans_vals.as<F>(), yhat, yhat,
                                      true, st, Role::Transfer);
    launch_colpanel_mrhs<F, F, double>(Bout.leaf_T, 0, Bout.leaf_T.ngroups(), rb, Bout.leaf_vals.as<F>(), yhat,
                                       yp, true, st, Role::Leaf);
    mark(4, st);
    if (ns == st) nearfield();
    join_side(op, ns, st);
    mark(7, st);
    launch_scatter_mrhs(Bout.perm_dev, nout, nb, rb, alpha, yp, ypn, y, ldy, st);
    mark(8, st);
}

// Work vectors of the operator for nrhs right-hand sides in blocks of rb.
static Work op_work(Op &op, int nrhs, int rb)
{
    if (nrhs == 1) return Work{op.xp.as<double>(), op.yp.as<double>(), op.ypn.as<double>(), op.xhat.p, op.yhat.p,
                               true, true, op.xt.as<double>(), op.yt.as<double>()};
    ensure_block_buffers(op, rb);
    return Work{op.xpb.as<double>(), op.ypb.as<double>(), op.ypbn.as<double>(), op.xhatb.p, op.yhatb.p, false,
                true, op.xtb.as<double>(), op.ytb.as<double>()};
}

// Layout of the work vectors for blocks of rb right-hand sides (rb = 1: one
// vector) in a buffer at base (NULL: sizes only); returns the bytes used.
static size_t work_layout(const Op &op, int rb, char *base, Work *w)
{
    const int64_t nmax = std::max(op.nrows, op.ncols);
    const int64_t hmax = std::max<int64_t>(std::max(op.rowb->hat_total, op.colb->hat_total), 1);
    const size_t fsz = basis_size(op.params.farfield_dtype);
    const int k = op.params.order_m * op.params.order_m * op.params.order_m;
    const int64_t kc = op.rowb->has_proj
                           ? (int64_t)k * std::max(op.rowb->tree->nclusters(), op.colb->tree->nclusters())
                           : 0;
    const size_t sizes[7] = {sizeof(double) * nmax * rb, sizeof(double) * nmax * rb, sizeof(double) * nmax * rb,
                             fsz * hmax * rb, fsz * hmax * rb, sizeof(double) * kc * rb, sizeof(double) * kc * rb};
    size_t off[7], at = 0;
    for (int i = 0; i < 7; ++i) {
        off[i] = at;
        at += (sizes[i] + 255) & ~size_t(255);
    }
    if (base && w)
        *w = Work{reinterpret_cast<double *>(base + off[0]), reinterpret_cast<double *>(base + off[1]),
                  reinterpret_cast<double *>(base + off[2]), base + off[3], base + off[4], false, false,
                  kc ? reinterpret_cast<double *>(base + off[5]) : nullptr,
                  kc ? reinterpret_cast<double *>(base + off[6]) : nullptr};
    return at;
}

template <typename F, typename C>
static void product(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y, int64_t ldy,
                    int nrhs, hipStream_t st, char *scratch_base)
{
    const int rb = nrhs == 1 ? 1 : block_width(op, nrhs);
    Work w{};
    if (scratch_base)
        work_layout(op, rb, scratch_base, &w);
    else
        w = op_work(op, nrhs, rb);
    if (nrhs == 1) {
        product_one<F, C>(op, w, trans, alpha, x, y, st);
        return;
    }
    for (int c = 0; c < nrhs; c += rb)
        product_block<F, C>(op, w, trans, alpha, x + c * ldx, ldx, y + c * ldy, ldy, std::min(rb, nrhs - c), rb,
                            st);
}

void check_product_args(const Op &op, int trans, const double *x, int64_t ldx, const double *y, int64_t ldy,
                        int nrhs)
{
    const int64_t nin = trans ? op.nrows : op.ncols;
    const int64_t nout = trans ? op.ncols : op.nrows;
    if (!x || !y) fail(H2B_EINVAL, "x and y must not be NULL");
    if (nrhs < 1 || nrhs > 64) fail(H2B_EINVAL, "nrhs must be in 1..64");
    if (ldx < nin || ldy < nout) fail(H2B_EINVAL, "leading dimension smaller than the vector length");
    {
        const char *xb = reinterpret_cast<const char *>(x);
        const char *yb = reinterpret_cast<const char *>(y);
        const char *xe = xb + sizeof(double) * (size_t)(ldx * (nrhs - 1) + nin);
        const char *ye = yb + sizeof(double) * (size_t)(ldy * (nrhs - 1) + nout);
        if (xb < ye && yb < xe) fail(H2B_EINVAL, "x and y overlap");
    }
}

void prepare_product(Op &op, int nrhs)
{
    if (nrhs > 1) ensure_block_buffers(op, block_width(op, nrhs));
}

void reserve_block_buffers(Op &op) { ensure_block_buffers(op, 64); }

static void dispatch_product(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y,
                             int64_t ldy, int nrhs, hipStream_t st, char *scratch_base)
{
    switch (op.params.farfield_dtype) {
    case H2B_F64: product<double, double>(op, trans, alpha, x, ldx, y, ldy, nrhs, st, scratch_base); break;
    case H2B_F32: product<float, float>(op, trans, alpha, x, ldx, y, ldy, nrhs, st, scratch_base); break;
    default: product<float, bf16_t>(op, trans, alpha, x, ldx, y, ldy, nrhs, st, scratch_base); break;
    }
}

void matvec(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y, int64_t ldy,
            int nrhs, hipStream_t st)
{
    check_product_args(op, trans, x, ldx, y, ldy, nrhs);
    dispatch_product(op, trans, alpha, x, ldx, y, ldy, nrhs, st, nullptr);
}

// ------------------------------------------- product without allocation
//
// Work vectors of h2b_matvec_noalloc: one file-scope device array per GPU,
// shared by every such call on that GPU.  Host code never uses the array's
// name as an address (on the host it names a stand-in, not device memory):
// the device address comes from hipGetSymbolAddress, once per device.

static __device__ __align__(256) unsigned char scratch[H2B_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::vector<char *> g_scratch_ptr;  // per device id; NULL until looked up
}  // namespace

static char *scratch_address()
{
    int dev = 0;
    hip_check(hipGetDevice(&dev), "current device");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (!ptr) fail(H2B_EDEVICE, "scratch symbol address is NULL");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    return g_scratch_ptr[dev];
}

void matvec_noalloc(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y, int64_t ldy,
                    int nrhs, hipStream_t st)
{
    check_product_args(op, trans, x, ldx, y, ldy, nrhs);
    const int rb = nrhs == 1 ? 1 : block_width(op, nrhs);
    const size_t need = work_layout(op, rb, nullptr, nullptr);
    if (need > (size_t)H2B_NOALLOC_SCRATCH_BYTES)
        fail(H2B_EINVAL, "the product needs " + std::to_string(need) + " bytes of work vectors, more than the " +
                             std::to_string((size_t)H2B_NOALLOC_SCRATCH_BYTES) + " of the static scratch array");
    dispatch_product(op, trans, alpha, x, ldx, y, ldy, nrhs, st, scratch_address());
}

// Autotuner of the many-right-hand-side coupling product: times every block
// width rb in {16, 32, 64} (and, on matrix cores, staging depth kc in {32, 64})
// on the operator's own coupling panels and keeps the fastest per column.
template <typename F, typename C>
static void tune_impl(Op &op, int nrhs, hipStream_t st, double *best_us)
{
    std::vector<std::pair<int, int>> cand;
    for (int rb : {16, 32, 64}) {
        if (rb > std::max(16, (nrhs + 15) / 16 * 16)) continue;
        if (std::is_same<F, float>::value)
            for (int kc : {32, 64}) cand.push_back({rb, kc});
        else
            cand.push_back({rb, 32});
    }
    ensure_block_buffers(op, 64);
    F *xh = op.xhatb.as<F>(), *yh = op.yhatb.as<F>();
    const int64_t hmax = std::max(op.rowb->hat_total, op.colb->hat_total);
    launch_fill_zero<F>(xh, hmax * 64, st);
    hipEvent_t e0, e1;
    hip_check(hipEventCreate(&e0), "event");
    hip_check(hipEventCreate(&e1), "event");
    double best = 1e300;
    for (auto &c : cand) {
        coupling_block<F, C>(op, 0, c.first, c.second, xh, yh, st);  // warm-up
        hip_check(hipEventRecord(e0, st), "event");
        for (int rep = 0; rep < 3; ++rep) coupling_block<F, C>(op, 0, c.first, c.second, xh, yh, st);
        hip_check(hipEventRecord(e1, st), "event");
        hip_check(hipEventSynchronize(e1), "event");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, e0, e1), "event");
        // time per right-hand side for nrhs columns processed in blocks of rb
        const int blocks = (nrhs + c.first - 1) / c.first;
        const double t = ms / 3.0 * blocks;
        if (t < best) {
            best = t;
            op.tune_rb = c.first;
            op.tune_kc = c.second;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (best_us) *best_us = best * 1e3;
}

void tune(Op &op, int nrhs, hipStream_t st, double *best_us)
{
    if (nrhs < 2 || nrhs > 64) fail(H2B_EINVAL, "nrhs must be in 2..64");
    switch (op.params.farfield_dtype) {
    case H2B_F64: tune_impl<double, double>(op, nrhs, st, best_us); break;
    case H2B_F32: tune_impl<float, float>(op, nrhs, st, best_us); break;
    default: tune_impl<float, bf16_t>(op, nrhs, st, best_us); break;
    }
}

// Mean milliseconds per recorded product of gather, forward, coupling,
// backward, nearfield (on the side stream, overlapping the far field),
// scatter, and the whole product.
void phase_times(Op &op, double out[7])
{
    if (op.nev == 0) fail(H2B_ESTATE, "no timed product recorded (enable timing first)");
    hip_check(hipEventSynchronize(op.ev[op.nev - 1][8]), "event sync");
    static const int from[7] = {0, 1, 2, 3, 5, 7, 0}, to[7] = {1, 2, 3, 4, 6, 8, 8};
    for (int i = 0; i < 7; ++i) out[i] = 0.0;
    for (size_t k = 0; k < op.nev; ++k)
        for (int i = 0; i < 7; ++i) {
            float ms = 0.f;
            hip_check(hipEventElapsedTime(&ms, op.ev[k][from[i]], op.ev[k][to[i]]), "event time");
            out[i] += ms;
        }
    for (int i = 0; i < 7; ++i) out[i] /= (double)op.nev;
    op.nev = 0;
}

void op_stats(const Op &op, h2b_op_stats &s)
{
    s = h2b_op_stats{};
    s.rows = op.nrows;
    s.cols = op.ncols;
    s.nfar = (int64_t)op.blocks->far_t.size();
    s.nnear = (int64_t)op.blocks->near_t.size();
    s.near_entries = op.near.total;
    s.coupling_entries = op.recompute ? 0 : op.cpl.total;
    s.coupling_evals = op.recompute ? op.cpl.total : 0;
    s.row_basis_entries = op.rowb->leaf.total + op.rowb->trans.total;
    s.col_basis_entries = (op.colb == op.rowb) ? 0 : op.colb->leaf.total + op.colb->trans.total;
    s.bytes_near = op.near.total * 8;
    s.bytes_far = s.coupling_entries * (int64_t)coupling_size(op.params.farfield_dtype) +
                  (s.row_basis_entries + s.col_basis_entries) * (int64_t)basis_size(op.params.farfield_dtype);
    if (op.rowb->has_proj)
        s.bytes_far += 8 * (op.rowb->proj.total + (op.colb == op.rowb ? 0 : op.colb->proj.total));
    s.bytes_vectors = (int64_t)(op.xp.bytes + op.yp.bytes + op.ypn.bytes + op.xhat.bytes + op.yhat.bytes +
                                op.xt.bytes + op.yt.bytes);
    if (op.sym) {
        s.near_sym_entries = op.sym->P.total;
        s.near_sym_columns = op.sym->col_base.back();
        s.near_sym_corrections = op.sym->ncorr;
    }
    if (op.symcpl) {
        s.cpl_sym_entries = op.symcpl->P.total;
        s.cpl_sym_columns = op.symcpl->col_base.back();
    }
    s.bytes_transposed = op.has_R ? op.near_R.total * 8 + (op.recompute ? 0 : op.cpl_R.total) *
                                                              (int64_t)coupling_size(op.params.farfield_dtype)
                                  : 0;
    s.row_coeffs = op.rowb->hat_total;
    s.col_coeffs = op.colb->hat_total;
    auto rk = [](const Basis &B, int32_t &mx, double &mean) {
        mx = 0;
        double sum = 0;
        for (int r : B.rank) {
            mx = std::max(mx, r);
            sum += r;
        }
        mean = B.rank.empty() ? 0.0 : sum / B.rank.size();
    };
    rk(*op.rowb, s.max_rank_row, s.mean_rank_row);
    rk(*op.colb, s.max_rank_col, s.mean_rank_col);
}

}  // namespace h2b

namespace h2b {

// ------------------------------------------------------ shape derivatives

void set_geometry(Op &op, const double *vx, const double *vy, const double *vz, hipStream_t st)
{
    if (!vx || !vy || !vz) fail(H2B_EINVAL, "vertex arrays must not be NULL");
    if (op.params.recompress_tol > 0.0 || op.params.gca_tol > 0.0)
        fail(H2B_ENOTSUP, "geometry updates keep the interpolation bases frozen; recompressed and "
                          "cross-approximation operators are not supported");
    const Mesh &M = *op.rowb->tree->mesh;
    const int64_t nv = M.nv, nt = M.nt;
    std::vector<double> nx(nt), ny(nt), nz(nt);
    for (int64_t v = 0; v < nv; ++v)
        if (!std::isfinite(vx[v]) || !std::isfinite(vy[v]) || !std::isfinite(vz[v]))
            fail(H2B_EINVAL, "non-finite vertex coordinate");
    for (int64_t i = 0; i < nt; ++i) {
        const int a = M.t0[i], b = M.t1[i], c = M.t2[i];
        const double e1[3] = {vx[b] - vx[a], vy[b] - vy[a], vz[b] - vz[a]};
        const double e2[3] = {vx[c] - vx[a], vy[c] - vy[a], vz[c] - vz[a]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(len > 0.0)) fail(H2B_EINVAL, "triangle " + std::to_string(i) + " has zero area");
        nx[i] = cr[0] / len;
        ny[i] = cr[1] / len;
        nz[i] = cr[2] / len;
    }
    auto up = [&](const double *src, const double *dst, int64_t n) {
        hip_check(hipMemcpyAsync(const_cast<double *>(dst), src, sizeof(double) * n, hipMemcpyHostToDevice, st),
                  "geometry upload");
    };
    up(vx, op.geo.vx, nv);
    up(vy, op.geo.vy, nv);
    up(vz, op.geo.vz, nv);
    up(nx.data(), op.geo.nx, nt);
    up(ny.data(), op.geo.ny, nt);
    up(nz.data(), op.geo.nz, nt);
    hip_check(hipStreamSynchronize(st), "geometry upload");
    QuadDev Qn = make_quad(op.params.q_near);
    assemble_near(op, Qn, st);
    std::vector<Basis *> bases{op.rowb.get()};
    if (op.colb != op.rowb) bases.push_back(op.colb.get());
    const int m = op.params.order_m;
    for (Basis *B : bases) {
        if (op.params.farfield_dtype == H2B_F64)
            assemble_basis<double>(*B, m, B->axes, op.geo, st);
        else
            assemble_basis<float>(*B, m, B->axes, op.geo, st);
        transpose_basis_values(*B, op.params.farfield_dtype, st);
    }
    hip_check(hipStreamSynchronize(st), "geometry assembly");
    if (op.has_R) make_transposed_copies(op, st);
    if (op.sym) make_symmetric_near(op, st);
}

// Leaf coefficients a(v) = backward transfers of S V^T v (the product
// stopped before the leaf bases), v already in cluster order.
template <typename F, typename C>
static void partial_product(Op &op, const double *vp, F *a, hipStream_t st)
{
    const Basis &B = *op.rowb;
    F *xhat = op.xhat.as<F>();
    forward<F>(B, vp, xhat, st);
    launch_fill_zero<F>(a, B.hat_total, st);
    bool done = false;
    if constexpr (std::is_same<F, double>::value) {
        if (op.recompute) {  // interpolation bases (no projections)
            recompute_coupling(op, 0, 1, xhat, a, nullptr, nullptr, st);
            done = true;
        }
    }
    if (!done)
        launch_rowpanel<C, F, F>(op.cpl, 0, op.cpl.ngroups(), op.cpl_vals.as<C>(), xhat, a, true, st,
                                 Role::Coupling);
    for (auto &s : B.bw_steps)
        launch_colpanel<F, F, F>(B.trans_T, s.first, s.second, B.trans_vals.as<F>(), a, a, st, Role::Transfer);
}

template <typename F, typename C>
static void shape_grad_impl(Op &op, const double *x, const double *y, double *gx, double *gy, double *gz,
                            hipStream_t st)
{
    const Basis &B = *op.rowb;
    const int64_t n = op.nrows;
    if (op.gxp.bytes < sizeof(double) * n) {
        op.gxp.alloc(sizeof(double) * n);
        op.gyp.alloc(sizeof(double) * n);
        op.gax.alloc(sizeof(F) * std::max<int64_t>(B.hat_total, 1));
        op.gay.alloc(sizeof(F) * std::max<int64_t>(B.hat_total, 1));
    }
    double *xp = op.gxp.as<double>(), *yp = op.gyp.as<double>();
    launch_gather(B.perm_dev, n, 1, x, n, xp, st);
    launch_gather(B.perm_dev, n, 1, y, n, yp, st);
    partial_product<F, C>(op, yp, op.gay.as<F>(), st);
    partial_product<F, C>(op, xp, op.gax.as<F>(), st);
    launch_near_grad(op.near, B.perm_dev, op.geo, make_quad(op.params.q_near), xp, yp, gx, gy, gz, st);
    launch_leaf_grad<F>(B.leaf, B.perm_dev, B.axes.as<double>(), op.params.order_m, op.geo,
                        make_quad(basis_quad_order(op.params.order_m)), op.gax.as<F>(), op.gay.as<F>(), xp, yp,
                        gx, gy, gz, st);
}

void slp_shape_grad(Op &op, const double *x, const double *y, double *gx, double *gy, double *gz,
                    hipStream_t st)
{
    if (op.kernel != H2B_SLP) fail(H2B_EINVAL, "the shape gradient is implemented for the single-layer matrix");
    if (op.params.recompress_tol > 0.0 || op.params.gca_tol > 0.0)
        fail(H2B_ENOTSUP, "the shape gradient needs the interpolation bases (recompress_tol = 0, gca_tol = 0)");
    if (!x || !y || !gx || !gy || !gz) fail(H2B_EINVAL, "NULL vector");
    switch (op.params.farfield_dtype) {
    case H2B_F64: shape_grad_impl<double, double>(op, x, y, gx, gy, gz, st); break;
    case H2B_F32: shape_grad_impl<float, float>(op, x, y, gx, gy, gz, st); break;
    default: shape_grad_impl<float, bf16_t>(op, x, y, gx, gy, gz, st); break;
    }
}

}  // namespace h2b
