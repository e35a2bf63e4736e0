// extern "C" boundary of the library: handle management, argument checks and
// translation of internal errors into h2b_status codes.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "hchol.hpp"
#include "op.hpp"

struct h2b_mesh_s {
    std::shared_ptr<h2b::Mesh> m;
};
struct h2b_tree_s {
    std::shared_ptr<h2b::Tree> t;
};
struct h2b_blocks_s {
    std::shared_ptr<h2b::Blocks> b;
};
struct h2b_op_s {
    std::unique_ptr<h2b::Op> op;
};
struct h2b_batch_s {
    std::unique_ptr<h2b::Batch> b;
};

namespace h2b {

namespace {
std::mutex g_alloc_mu;
DeviceAllocator g_alloc;
thread_local hipStream_t g_alloc_stream = nullptr;
}  // namespace

DeviceAllocator current_allocator()
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

void set_allocator(const DeviceAllocator &a)
{
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc = a;
}

hipStream_t alloc_stream() { return g_alloc_stream; }

AllocStreamScope::AllocStreamScope(hipStream_t st) : saved(g_alloc_stream) { g_alloc_stream = st; }
AllocStreamScope::~AllocStreamScope() { g_alloc_stream = saved; }

}  // namespace h2b

namespace {

thread_local std::string g_err;

template <typename F> h2b_status guarded(F &&f)
{
    try {
        f();
        g_err.clear();
        return H2B_OK;
    } catch (const h2b::Error &e) {
        g_err = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host allocation failed";
        return H2B_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return H2B_EINVAL;
    } catch (...) {
        g_err = "unknown error";
        return H2B_EINVAL;
    }
}

void need(const void *p, const char *what)
{
    if (!p) h2b::fail(H2B_EINVAL, std::string(what) + " is NULL");
}

}  // namespace

extern "C" {

const char *h2b_last_error(void) { return g_err.c_str(); }

h2b_status h2b_set_allocator(h2b_alloc_fn alloc, h2b_free_fn free, void *ctx)
{
    return guarded([&] {
        if ((alloc == nullptr) != (free == nullptr))
            h2b::fail(H2B_EINVAL, "alloc and free must both be set or both be NULL");
        h2b::DeviceAllocator a;
        a.alloc = alloc;
        a.free = free;
        a.ctx = alloc ? ctx : nullptr;
        h2b::set_allocator(a);
    });
}

const char *h2b_version(void) { return "h2bem 0.1 (gfx950)"; }

h2b_status h2b_mesh_create(int64_t nv, const double *vx, const double *vy, const double *vz,
                           int64_t nt, const int32_t *t0, const int32_t *t1, const int32_t *t2,
                           h2b_mesh *out)
{
    return guarded([&] {
        need(out, "out");
        auto h = new h2b_mesh_s{h2b::make_mesh(nv, vx, vy, vz, nt, t0, t1, t2)};
        *out = h;
    });
}

h2b_status h2b_mesh_destroy(h2b_mesh mesh)
{
    delete mesh;
    return H2B_OK;
}

h2b_status h2b_tree_build(h2b_mesh mesh, h2b_space space, int leaf_size, h2b_tree *out)
{
    return guarded([&] {
        need(mesh, "mesh");
        need(out, "out");
        auto t = h2b::build_tree(mesh->m, space, leaf_size);
        *out = new h2b_tree_s{t};
    });
}

h2b_status h2b_tree_destroy(h2b_tree tree)
{
    delete tree;
    return H2B_OK;
}

h2b_status h2b_tree_info(h2b_tree tree, int64_t *n, int64_t *nclusters, int64_t *nleaves,
                         int32_t *nlevels)
{
    return guarded([&] {
        need(tree, "tree");
        const auto &T = *tree->t;
        if (n) *n = T.n;
        if (nclusters) *nclusters = T.nclusters();
        if (nleaves) *nleaves = (int64_t)T.leaves.size();
        if (nlevels) *nlevels = T.nlevels;
    });
}

h2b_status h2b_tree_arrays(h2b_tree tree, int32_t *perm, int32_t *begin, int32_t *end,
                           int32_t *parent, double *box)
{
    return guarded([&] {
        need(tree, "tree");
        const auto &T = *tree->t;
        if (perm) std::memcpy(perm, T.perm.data(), sizeof(int32_t) * T.perm.size());
        if (begin) std::memcpy(begin, T.begin.data(), sizeof(int32_t) * T.begin.size());
        if (end) std::memcpy(end, T.end.data(), sizeof(int32_t) * T.end.size());
        if (parent) std::memcpy(parent, T.parent.data(), sizeof(int32_t) * T.parent.size());
        if (box) std::memcpy(box, T.box.data(), sizeof(double) * T.box.size());
    });
}

h2b_status h2b_tree_gca(h2b_tree tree, int order_m, double eps, int32_t *ranks, int32_t *pivots,
                        int64_t *npivots)
{
    return guarded([&] {
        need(tree, "tree");
        need(ranks, "ranks");
        if (order_m < 1 || order_m > h2b::MMAX) h2b::fail(H2B_EINVAL, "order_m must be in 1..6");
        if (!(eps > 0.0) || !std::isfinite(eps)) h2b::fail(H2B_EINVAL, "eps must be finite and > 0");
        const h2b::GcaBases G = h2b::gca_bases(*tree->t, order_m, eps);
        int64_t k = 0;
        for (size_t c = 0; c < G.rank.size(); ++c) {
            ranks[c] = G.rank[c];
            if (pivots)
                for (int32_t p : G.hat[c]) pivots[k++] = p;
        }
        if (npivots) *npivots = k;
    });
}

h2b_status h2b_blocks_build(h2b_tree rows, h2b_tree cols, double eta, int far_disabled,
                            h2b_blocks *out)
{
    return guarded([&] {
        need(rows, "rows");
        need(cols, "cols");
        need(out, "out");
        auto b = h2b::build_blocks(rows->t, cols->t, eta, far_disabled != 0);
        *out = new h2b_blocks_s{b};
    });
}

h2b_status h2b_blocks_destroy(h2b_blocks blocks)
{
    delete blocks;
    return H2B_OK;
}

h2b_status h2b_blocks_info(h2b_blocks blocks, int64_t *nfar, int64_t *nnear, int64_t *near_entries)
{
    return guarded([&] {
        need(blocks, "blocks");
        const auto &B = *blocks->b;
        if (nfar) *nfar = (int64_t)B.far_t.size();
        if (nnear) *nnear = (int64_t)B.near_t.size();
        if (near_entries) {
            int64_t s = 0;
            for (size_t i = 0; i < B.near_t.size(); ++i)
                s += (int64_t)B.rows->size(B.near_t[i]) * B.cols->size(B.near_s[i]);
            *near_entries = s;
        }
    });
}

h2b_status h2b_blocks_lists(h2b_blocks blocks, int32_t *far_pairs, int32_t *near_pairs)
{
    return guarded([&] {
        need(blocks, "blocks");
        const auto &B = *blocks->b;
        if (far_pairs)
            for (size_t i = 0; i < B.far_t.size(); ++i) {
                far_pairs[2 * i] = B.far_t[i];
                far_pairs[2 * i + 1] = B.far_s[i];
            }
        if (near_pairs)
            for (size_t i = 0; i < B.near_t.size(); ++i) {
                near_pairs[2 * i] = B.near_t[i];
                near_pairs[2 * i + 1] = B.near_s[i];
            }
    });
}

void h2b_params_default(h2b_params *p)
{
    if (!p) return;
    p->order_m = 4;
    p->q_near = 4;
    p->recompress_tol = 0.0;
    p->farfield_dtype = H2B_F64;
    p->transposed_copy = 1;
    p->symmetric_near = 1;
    p->gca_tol = 0.0;
    p->recompute_coupling = 0;
}

h2b_status h2b_assemble(h2b_blocks blocks, h2b_kernel kernel, const h2b_params *params,
                        void *hip_stream, h2b_op *out)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(blocks, "blocks");
        need(params, "params");
        need(out, "out");
        auto op = h2b::assemble_op(blocks->b, kernel, *params, static_cast<hipStream_t>(hip_stream));
        *out = new h2b_op_s{std::move(op)};
    });
}

h2b_status h2b_op_destroy(h2b_op op)
{
    delete op;
    return H2B_OK;
}

h2b_status h2b_op_info(h2b_op op, h2b_op_stats *out)
{
    return guarded([&] {
        need(op, "op");
        need(out, "out");
        h2b::op_stats(*op->op, *out);
    });
}

h2b_status h2b_matvec(h2b_op op, int trans, double alpha, const double *x, int64_t ldx, double *y,
                      int64_t ldy, int nrhs, void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(op, "op");
        h2b::matvec(*op->op, trans ? 1 : 0, alpha, x, ldx, y, ldy, nrhs,
                    static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_matvec_noalloc(h2b_op op, int trans, double alpha, const double *x, int64_t ldx, double *y,
                              int64_t ldy, int nrhs, void *hip_stream)
{
    return guarded([&] {
        need(op, "op");
        h2b::matvec_noalloc(*op->op, trans ? 1 : 0, alpha, x, ldx, y, ldy, nrhs,
                            static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_batch_create(int nops, const h2b_op *ops, const int *trans, const double *alpha,
                            const double *const *x, const int64_t *ldx, double *const *y,
                            const int64_t *ldy, const int *nrhs, void *hip_stream, h2b_batch *out)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(ops, "ops");
        need(out, "out");
        std::vector<h2b::Op *> raw(nops > 0 ? nops : 0);
        for (int i = 0; i < nops; ++i) {
            need(ops[i], "ops[i]");
            raw[i] = ops[i]->op.get();
        }
        auto b = h2b::batch_create(nops, raw.data(), trans, alpha, x, ldx, y, ldy, nrhs,
                                   static_cast<hipStream_t>(hip_stream));
        *out = new h2b_batch_s{std::move(b)};
    });
}

h2b_status h2b_batch_launch(h2b_batch batch, void *hip_stream)
{
    return guarded([&] {
        need(batch, "batch");
        h2b::batch_launch(*batch->b, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_batch_destroy(h2b_batch batch)
{
    delete batch;
    return H2B_OK;
}

h2b_status h2b_op_tune(h2b_op op, int nrhs, void *hip_stream, double *best_us)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(op, "op");
        h2b::tune(*op->op, nrhs, static_cast<hipStream_t>(hip_stream), best_us);
    });
}

h2b_status h2b_op_set_geometry(h2b_op op, const double *vx, const double *vy, const double *vz,
                               void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(op, "op");
        h2b::set_geometry(*op->op, vx, vy, vz, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_slp_shape_grad(h2b_op G, const double *x, const double *y, double *gvx, double *gvy,
                              double *gvz, void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(G, "G");
        h2b::slp_shape_grad(*G->op, x, y, gvx, gvy, gvz, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_slp_bilinear(h2b_op G, const double *x, const double *y, double *gy, double *out,
                            void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(G, "G");
        h2b::slp_bilinear(*G->op, x, y, gy, out, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_op_set_timing(h2b_op op, int enable)
{
    return guarded([&] {
        need(op, "op");
        op->op->timing = enable != 0;
        op->op->nev = 0;
    });
}

h2b_status h2b_op_set_overlap(h2b_op op, int enable)
{
    return guarded([&] {
        need(op, "op");
        op->op->overlap = enable != 0;
    });
}

h2b_status h2b_op_phase_times(h2b_op op, double phases_ms[7])
{
    return guarded([&] {
        need(op, "op");
        need(phases_ms, "phases_ms");
        h2b::phase_times(*op->op, phases_ms);
    });
}

void h2b_cg_params_default(h2b_cg_params *p)
{
    if (!p) return;
    p->tol = 1e-8;
    p->max_iter = 1000;
    p->check_every = 8;
    p->use_graph = 1;
    p->zero_guess = 1;
    p->form = H2B_FORM_PRODUCT;
    p->precond = H2B_PRECOND_NONE;
    p->hchol = nullptr;
}

h2b_status h2b_hchol_build(h2b_op G, double eps, h2b_hchol *out, void *hip_stream)
{
    return guarded([&] {
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        h2b::AllocStreamScope scope(st);
        need(G, "G");
        need(out, "out");
        if (!(eps >= 0.0) || !std::isfinite(eps)) h2b::fail(H2B_EINVAL, "eps must be finite and >= 0");
        auto P = std::make_unique<h2b::HChol>();
        P->eps = eps;
        auto t0 = std::chrono::steady_clock::now();
        P->H = h2b::hmatrix_from_op(*G->op, eps, st);
        P->convert_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        h2b::hchol_factor(*P, eps);
        t0 = std::chrono::steady_clock::now();
        h2b::hchol_upload(*P, st);
        P->upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = new h2b_hchol_s{std::move(P)};
    });
}

h2b_status h2b_hchol_from_dense(h2b_blocks blocks, const double *A, double eps, h2b_hchol *out)
{
    return guarded([&] {
        need(blocks, "blocks");
        need(A, "A");
        need(out, "out");
        if (!(eps >= 0.0) || !std::isfinite(eps)) h2b::fail(H2B_EINVAL, "eps must be finite and >= 0");
        const h2b::Blocks &B = *blocks->b;
        if (B.rows != B.cols) h2b::fail(H2B_EINVAL, "the blocks must be on one cluster tree");
        const h2b::Tree &T = *B.rows;
        const int64_t n = T.n;
        std::vector<double> Ap((size_t)n * n);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = 0; j < n; ++j) Ap[(size_t)i * n + j] = A[(size_t)T.perm[i] * n + T.perm[j]];
        auto P = std::make_unique<h2b::HChol>();
        P->eps = eps;
        auto t0 = std::chrono::steady_clock::now();
        P->H = h2b::hmatrix_from_dense(B, Ap.data(), eps);
        P->convert_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        h2b::hchol_factor(*P, eps);
        *out = new h2b_hchol_s{std::move(P)};
    });
}

h2b_status h2b_hchol_solve_host(h2b_hchol P, const double *r, double *z)
{
    return guarded([&] {
        need(P, "P");
        need(r, "r");
        need(z, "z");
        const h2b::Tree &T = *P->p->H->tree;
        std::vector<double> x((size_t)T.n);
        for (int64_t i = 0; i < T.n; ++i) x[i] = r[T.perm[i]];
        h2b::hchol_flatten(*P->p);
        h2b::hprogram_run(P->p->prog_host, T.n, x.data());
        for (int64_t i = 0; i < T.n; ++i) z[T.perm[i]] = x[i];
    });
}

h2b_status h2b_hchol_apply(h2b_hchol P, const double *r, double *z, void *hip_stream)
{
    return guarded([&] {
        const hipStream_t st = static_cast<hipStream_t>(hip_stream);
        h2b::AllocStreamScope scope(st);
        need(P, "P");
        need(r, "r");
        need(z, "z");
        const int64_t n = P->p->H->tree->n;
        const char *rb = reinterpret_cast<const char *>(r), *zb = reinterpret_cast<const char *>(z);
        if (rb < zb + sizeof(double) * n && zb < rb + sizeof(double) * n) h2b::fail(H2B_EINVAL, "r and z overlap");
        if (!P->p->uploaded) {
            const auto t0 = std::chrono::steady_clock::now();
            h2b::hchol_upload(*P->p, st);
            P->p->upload_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        }
        h2b::hchol_apply(*P->p, r, z, st);
    });
}

h2b_status h2b_hchol_get_info(h2b_hchol P, h2b_hchol_info *info)
{
    return guarded([&] {
        need(P, "P");
        need(info, "info");
        const h2b::HChol &H = *P->p;
        h2b_hchol_info o{};
        o.n = H.H->tree->n;
        o.eps = H.eps;
        o.coarse_entries = H.coarse.dense_entries + H.coarse.rk_entries;
        o.dense_entries = H.factor.dense_entries;
        o.rk_entries = H.factor.rk_entries;
        o.dense_blocks = H.factor.dense_blocks;
        o.rk_blocks = H.factor.rk_blocks;
        o.max_rank = H.factor.max_rank;
        o.coarsened_blocks = H.factor.coarsened;
        o.converted_blocks = H.factor.converted;
        o.steps = H.nsteps;
        o.tasks = H.ntasks;
        o.convert_s = H.convert_s;
        o.coarsen_s = H.coarsen_s;
        o.factor_s = H.factor_s;
        o.upload_s = H.upload_s;
        *info = o;
    });
}

h2b_status h2b_hchol_destroy(h2b_hchol P)
{
    return guarded([&] {
        if (P && P->p && P->p->uploaded) (void)hipDeviceSynchronize();
        delete P;
    });
}

h2b_status h2b_hypersingular_matvec(h2b_op G, double alpha, const double *x, double *y, void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(G, "G");
        h2b::hypersingular_matvec(*G->op, alpha, x, y, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_mass_matvec(h2b_op op, int trans, double alpha, const double *x, double *y, void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(op, "op");
        h2b::mass_matvec(*op->op, trans ? 1 : 0, alpha, x, y, static_cast<hipStream_t>(hip_stream));
    });
}

h2b_status h2b_cg_solve(h2b_op A, const double *b, double *x, const h2b_cg_params *params,
                        h2b_cg_result *result, double *history, void *hip_stream)
{
    return guarded([&] {
        h2b::AllocStreamScope scope(static_cast<hipStream_t>(hip_stream));
        need(A, "A");
        need(params, "params");
        need(result, "result");
        h2b_cg_result r{};
        h2b::cg_solve(*A->op, b, x, *params, r, history, static_cast<hipStream_t>(hip_stream));
        *result = r;
    });
}

}  // extern "C"
