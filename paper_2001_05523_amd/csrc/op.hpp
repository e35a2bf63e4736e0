// Assembled H^2 operator and its product driver.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <memory>
#include <utility>
#include <vector>

#include "device.hpp"

namespace h2b {

// Work descriptors of the single-vector basis transformations (transform.hip):
// one per cluster with coefficients, the leaves first, then the parents by
// level from the deepest; step[k] .. step[k + 1] is one launch.
struct LevelDescs {
    std::vector<int32_t> desc, step;
    const int32_t *d_desc = nullptr;
    DevMem mem;
};

// Cluster basis on one tree: leaf matrices (stored transposed) and transfer
// matrices, each with the panel descriptors of the forward (rows) and the
// backward (transposed) products.
struct Basis {
    std::shared_ptr<const Tree> tree;
    bool dlp_cols = false;                  // normal-derivative basis of the P1 space
    std::vector<int32_t> rank;              // k_t per cluster
    std::vector<int64_t> hat_off;           // offset of cluster coefficients
    int64_t hat_total = 0;
    RowPanels leaf;                         // V_t^T per leaf
    ColPanels leaf_T;
    RowPanels trans;                        // [E_c0^T | E_c1^T] per parent, deepest level first
    ColPanels trans_T;
    std::vector<std::pair<int, int>> fw_steps;  // group ranges of trans, bottom-up
    std::vector<std::pair<int, int>> bw_steps;  // group ranges of trans_T, top-down
    DevMem leaf_vals, trans_vals;
    // forward transformation as column products over transposed copies
    ColPanels leaf_F, trans_F;              // one output group per row-panel group
    DevMem leafT_vals, transT_vals;
    DevMem axes;                            // Chebyshev points, 3*m per cluster
    DevMem perm_mem;
    const int32_t *perm_dev = nullptr;
    // Coupling evaluated on the fly after recompression: P_c (k'_c x k) per
    // cluster, rows at the cluster's coefficients, columns at c * k of the
    // interpolation coefficients.
    RowPanels proj;
    ColPanels proj_T;
    DevMem proj_vals;
    bool has_proj = false;
    std::unique_ptr<LevelDescs> lev;        // descriptors of the single-vector transformations
};

// Nearfield of G on one cluster tree stored once per pair of leaves: for every
// row leaf t the panel [N_tt | N_ts for the nearfield leaves s > t].  The
// product reads each off-diagonal block once for both y_t += N_ts x_s and
// y_s += N_ts^T x_t; the column sums go to `colsum` and are added per leaf by
// a second launch, which also applies the sparse correction of the touching
// pairs across leaves, whose two quadratures agree only to quadrature error
// (G_ji - G_ij, stored for G x by row j and for G^T x by row i).
struct SymNear {
    RowPanels P;                    // groups = row leaves, segment 0 = the diagonal block
    DevMem vals;
    DevMem colsum;                  // one column sum per panel column
    std::vector<int64_t> col_base;  // first colsum entry of each group
    ColPanels red;                  // per leaf u: the blocks (t, u), t != u, as colsum offsets
    // copy of the stored blocks out of the full nearfield
    std::vector<int64_t> cp_src, cp_dst;
    std::vector<int32_t> cp_src_ld, cp_dst_ld, cp_rows, cp_cols;
    // corrections: CSR over cluster-ordered rows, for G x (fwd) and G^T x (bwd)
    std::vector<int64_t> cf_ptr, cb_ptr;
    std::vector<int32_t> cf_idx, cb_idx;
    std::vector<int64_t> cf_a, cf_b, cb_a, cb_b;  // value = near[a] - near[b]
    DevMem desc, cf_val, cb_val;
    const int64_t *d_col_base = nullptr, *d_cp_src = nullptr, *d_cp_dst = nullptr;
    const int32_t *d_cp_src_ld = nullptr, *d_cp_dst_ld = nullptr, *d_cp_rows = nullptr, *d_cp_cols = nullptr;
    const int64_t *d_cf_ptr = nullptr, *d_cb_ptr = nullptr, *d_cf_a = nullptr, *d_cf_b = nullptr;
    const int64_t *d_cb_a = nullptr, *d_cb_b = nullptr;
    const int32_t *d_cf_idx = nullptr, *d_cb_idx = nullptr;
    int64_t ncorr = 0;
};

constexpr int SYMCPL_MAX_RANK = 256;  // largest cluster rank of the once-per-pair coupling

// Far field of G stored once per pair of clusters: for every row cluster t
// the panel [S_ts for the farfield clusters s > t] (S_st = S_ts^T, one basis
// for rows and columns).  One pass adds the row sums to y^_t and writes the
// column sums S_ts^T x^_t to `colsum`; a second launch adds those per cluster.
struct SymCpl {
    RowPanels P;                    // groups = row clusters, segments = farfield clusters s > t
    DevMem vals;
    DevMem colsum;                  // one column sum per panel column
    std::vector<int64_t> col_base;  // first colsum entry of each group
    ColPanels red;                  // per cluster u: the blocks (t, u), t < u, as colsum offsets
    std::vector<int64_t> cp_src, cp_dst;  // copy of the stored blocks out of the full coupling panels
    std::vector<int32_t> cp_src_ld, cp_dst_ld, cp_rows, cp_cols;
    DevMem desc;
    const int64_t *d_col_base = nullptr, *d_cp_src = nullptr, *d_cp_dst = nullptr;
    const int32_t *d_cp_src_ld = nullptr, *d_cp_dst_ld = nullptr, *d_cp_rows = nullptr, *d_cp_cols = nullptr;
    bool f32 = false;               // values and column sums in FP32 (FP32 far field), else FP64
};

struct Op {
    std::shared_ptr<const Blocks> blocks;
    h2b_kernel kernel = H2B_SLP;
    h2b_params params{};
    int64_t nrows = 0, ncols = 0;
    std::shared_ptr<Basis> rowb, colb;      // colb == rowb for G
    GeoDev geo{};
    DevMem geo_mem;
    RowPanels near;
    ColPanels near_T;
    DevMem near_vals;
    RowPanels cpl;
    ColPanels cpl_T;
    DevMem cpl_vals;
    // Transposed copies grouped by column cluster (params.transposed_copy):
    // A^T x then runs the row-panel kernels.
    RowPanels near_R, cpl_R;
    DevMem near_R_vals, cpl_R_vals;
    bool has_R = false;
    std::unique_ptr<SymNear> sym;           // params.symmetric_near for G on one tree
    std::unique_ptr<SymCpl> symcpl;         // the same for G's stored FP64 or FP32 coupling
    DevMem xp, yp, xhat, yhat;              // product work vectors
    DevMem ypn;                             // near-field output (summed with yp by the scatter)
    DevMem xpb, ypb, xhatb, yhatb, ypbn;    // block work vectors (many right-hand sides)
    // params.recompute_coupling: no coupling values are stored; the coupling
    // product evaluates S_ts (cpl / cpl_R give the blocks with rank-k
    // offsets), through the interpolation coefficients xt, yt (k per cluster)
    // when the bases were recompressed
    bool recompute = false;
    DevMem xt, yt, xtb, ytb;
    // The near field runs on its own stream beside the far field: forked
    // after the gather, joined before the scatter.
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    bool overlap = true;                    // false: the nearfield stays on the caller's stream
    DevMem gxp, gyp, gax, gay;              // shape-gradient work vectors
    DevMem hs_c, hs_g;                      // hypersingular product: curls and G times curls (3 nt each)
    // block-Jacobi preconditioner (built by the first preconditioned solve):
    // per leaf its first position, size and the offset of its inverse block
    DevMem bj_inv, bj_mem;
    const int32_t *bj_begin = nullptr, *bj_n = nullptr;
    const int64_t *bj_dst = nullptr;
    int bj_leaves = 0;
    int mrhs_rb = 0;                        // block width the block vectors are sized for
    int tune_rb = 0, tune_kc = 32;          // autotuned coupling tile (0: not tuned)
    bool timing = false;
    std::vector<std::array<hipEvent_t, 9>> ev;  // one event set per timed product
    size_t nev = 0;                              // timed products since timing was enabled
    ~Op();
};

// Element sizes of the far-field storage for a far-field dtype.
inline size_t basis_size(h2b_dtype dt) { return dt == H2B_F64 ? sizeof(double) : sizeof(float); }
inline size_t coupling_size(h2b_dtype dt)
{
    return dt == H2B_F64 ? sizeof(double) : dt == H2B_F32 ? sizeof(float) : sizeof(bf16_t);
}

QuadDev make_quad(int q);

// Basis values (in the far-field dtype) and coupling entries A|_{t_hat x s_hat}
// of an operator whose panels were built with the GCA ranks (Gr: row tree,
// Gc: column tree, the same object for G).
void set_gca_values(Op &op, const GcaBases &Gr, const GcaBases &Gc, hipStream_t st);

std::unique_ptr<Op> assemble_op(std::shared_ptr<const Blocks> blocks, h2b_kernel kernel,
                                const h2b_params &p, hipStream_t st);
void build_basis_structure(Basis &B, const std::vector<int> &ranks, hipStream_t st);
// Subtree schedule of a basis (from its final panels).
void build_level_descriptors(Basis &B, hipStream_t st);
template <typename F> void forward_levels(const Basis &B, const double *xp, F *xhat, hipStream_t st);
template <typename F> void backward_levels(const Basis &B, F *yhat, double *yp, hipStream_t st);
// Transposed copies of the leaf and transfer values (after they are final).
void transpose_basis_values(Basis &B, h2b_dtype dt, hipStream_t st);
void recompress_op(Op &op, double tol, hipStream_t st);
// Coupling evaluated on the fly: structure of the transposed grouping.
void setup_recompute(Op &op, hipStream_t st);
// Projections P_c of a recompressed basis for the evaluated coupling.
void set_projection(Basis &B, int k, const std::vector<std::vector<double>> &P, hipStream_t st);
// yhat += op(S) xhat over every farfield block, S evaluated; rb = 1 or the
// block width; xt, yt: interpolation-coefficient work vectors (projections only).
void recompute_coupling(const Op &op, int trans, int rb, const double *xhat, double *yhat, double *xt, double *yt,
                        hipStream_t st);
// (Re)builds the transposed copies from the current nearfield and coupling values.
void make_transposed_copies(Op &op, hipStream_t st);
// Structure (first call) and values of the once-per-pair nearfield of G.
void make_symmetric_near(Op &op, hipStream_t st);
// ypn += N x (trans = 0) or N^T x (trans = 1) from the once-per-pair storage.
void symmetric_near_product(const Op &op, int trans, const double *xp, double *ypn, hipStream_t st);
// Structure (first call) and values of the once-per-pair coupling of G.
void make_symmetric_coupling(Op &op, hipStream_t st);
// yhat += S xhat (= S^T xhat) from the once-per-pair coupling (T: the far-field precision).
template <typename T> void symmetric_coupling_product(const Op &op, const T *xhat, T *yhat, hipStream_t st);
void check_product_args(const Op &op, int trans, const double *x, int64_t ldx, const double *y, int64_t ldy,
                        int nrhs);
// Allocates what a product with nrhs right-hand sides needs (before a capture).
void prepare_product(Op &op, int nrhs);
// Block work vectors at the widest block (64 columns): a graph that captured
// them stays valid, since no later product or tuning has to reallocate them.
void reserve_block_buffers(Op &op);
void matvec(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y, int64_t ldy,
            int nrhs, hipStream_t st);
// The same product with its work vectors in the static scratch array (no allocation).
void matvec_noalloc(Op &op, int trans, double alpha, const double *x, int64_t ldx, double *y, int64_t ldy,
                    int nrhs, hipStream_t st);
// Nodes the next work captured on st will depend on, and their replacement
// (st must be capturing): with these a single captured stream forms parallel
// branches of the graph.
std::vector<hipGraphNode_t> capture_tail(hipStream_t st);
void set_capture_tail(hipStream_t st, std::vector<hipGraphNode_t> deps);

// Merged batch: one launch per step for all operators (batch_merged.hip).
struct MergedBatch;
struct MergedBatchDeleter {
    void operator()(MergedBatch *m) const;
};
using MergedPtr = std::unique_ptr<MergedBatch, MergedBatchDeleter>;
// NULL if the products cannot share one program (different far-field types,
// directions or numbers of right-hand sides, evaluated couplings, A^T x
// without transposed copies).
MergedPtr merged_create(int nops, Op *const *ops, const int *trans, const double *alpha, const double *const *x,
                        const int64_t *ldx, double *const *y, const int64_t *ldy, const int *nrhs, hipStream_t st);
// Queues the merged products on st (which must be capturing).
void merged_capture(MergedBatch &m, hipStream_t st);
int64_t merged_launches(const MergedBatch &m);

// A captured batch of products (one graph, one forked stream per operator).
struct Batch {
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    MergedPtr merged;  // the merged program, or NULL for a graph of per-operator products
    ~Batch();
};
std::unique_ptr<Batch> batch_create(int nops, Op *const *ops, const int *trans, const double *alpha,
                                    const double *const *x, const int64_t *ldx, double *const *y,
                                    const int64_t *ldy, const int *nrhs, hipStream_t st);
void batch_launch(Batch &b, hipStream_t st);
void phase_times(Op &op, double out[7]);
void tune(Op &op, int nrhs, hipStream_t st, double *best_us);
// Re-assembles the geometry-dependent parts (near field, leaf bases) for new
// vertex coordinates with trees, boxes and interpolation points frozen.
void set_geometry(Op &op, const double *vx, const double *vy, const double *vz, hipStream_t st);
// (gx, gy, gz) += d(x^T G y)/d(vertex coordinates) for the frozen structure.
void slp_shape_grad(Op &op, const double *x, const double *y, double *gx, double *gy, double *gz,
                    hipStream_t st);
void op_stats(const Op &op, h2b_op_stats &s);
// y += alpha M x (trans = 0) or alpha M^T x (trans = 1), M the mixed mass matrix.
void mass_matvec(Op &op, int trans, double alpha, const double *x, double *y, hipStream_t st);
// y += alpha W x, W = sum_d C_d^T G C_d the hypersingular matrix from G.
void hypersingular_matvec(Op &G, double alpha, const double *x, double *y, hipStream_t st);
// Allocates what hypersingular_matvec needs (before a capture).
void prepare_hypersingular(Op &G);
// gy = G y and *out = x^T gy (device scalar), the single-layer bilinear form.
void slp_bilinear(Op &G, const double *x, const double *y, double *gy, double *out, hipStream_t st);
// Conjugate gradients for A x = b with the H^2 product of A (or W x = b).
void cg_solve(Op &A, const double *b, double *x, const h2b_cg_params &prm, h2b_cg_result &res, double *history,
              hipStream_t st);

}  // namespace h2b
