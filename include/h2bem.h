/*
 * h2bem.h -- C interface of the MI355X (gfx950) H^2-matrix boundary element
 * library for the 3-D Laplace equation.
 *
 * The library builds cluster and block trees for a flat triangle mesh,
 * assembles the Galerkin single-layer matrix G and double-layer matrix K in
 * H^2 form (interpolation far field, regularised-quadrature near field), and
 * multiplies them with vectors on the GPU:
 *
 *   G (I x I): g_ij = int psi_i(x) int g(x,y) psi_j(y) dy dx       (paper, Section 1, eq. (slp))
 *   K (I x J): k_ij = int psi_i(x) int dg/dn_y(x,y) phi_j(y) dy dx (paper, Section 1, eq. (dlp))
 *   g(x,y) = 1 / (4 pi |x - y|)                                    (paper, Section 1)
 *
 * psi_i is the indicator of triangle i (index set I = triangles) and phi_j the
 * continuous piecewise-linear hat function of vertex j (index set J =
 * vertices), the discrete spaces chosen in Section 5.
 *
 * Conventions
 *  - Every function returns an h2b_status; h2b_last_error() gives a message for
 *    the last failing call on the calling thread.  No C++ exception crosses
 *    this interface.  On error no output handle is written and no vector is
 *    modified.
 *  - Mesh arrays are host memory and are copied.  Vectors passed to the
 *    products are device memory owned by the caller and are used
 *    asynchronously on the given HIP stream (hipStream_t passed as void*; NULL
 *    = the default stream); they must stay valid until the stream has passed
 *    the call.  Vectors use the caller's numbering (triangle order for I,
 *    vertex order for J); the cluster permutation is internal.
 *  - Handles own their data.  A handle keeps alive everything it was built from
 *    (an operator keeps its blocks, trees and mesh), so handles may be
 *    destroyed in any order.
 *  - Calls on one operator must not overlap in time on different streams: the
 *    operator owns the intermediate vectors of its products.
 */
#ifndef H2BEM_H
#define H2BEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    H2B_OK = 0,
    H2B_EINVAL = -1,   /* invalid argument (checked on the host before any launch) */
    H2B_ENOMEM = -2,   /* host or device allocation failed */
    H2B_EDEVICE = -3,  /* a HIP call failed */
    H2B_ESTATE = -4,   /* handle in the wrong state for this call */
    H2B_ENOTSUP = -5   /* valid request the library does not support */
} h2b_status;

typedef enum { H2B_P0 = 0, H2B_P1 = 1 } h2b_space;        /* triangles (I) / vertices (J) */
typedef enum { H2B_SLP = 0, H2B_DLP = 1 } h2b_kernel;     /* G (P0 x P0) / K (P0 x P1) */
/* Far-field storage: F64 everything double; F32 bases, coupling matrices and
 * cluster coefficients float with float accumulation; BF16 as F32 but the
 * coupling matrices stored in bfloat16.  The near field is always double. */
typedef enum { H2B_F64 = 0, H2B_F32 = 1, H2B_BF16 = 2 } h2b_dtype;

typedef struct h2b_mesh_s *h2b_mesh;
typedef struct h2b_tree_s *h2b_tree;
typedef struct h2b_blocks_s *h2b_blocks;
typedef struct h2b_op_s *h2b_op;
typedef struct h2b_batch_s *h2b_batch;

/* ------------------------------------------------------ device memory */

/* Device allocator callbacks.  alloc returns `bytes` of device memory on the
 * current HIP device (aligned to at least 256 bytes), or NULL if it cannot;
 * hip_stream is the stream of the library call that asks (NULL for the
 * default stream), ctx the pointer given to h2b_set_allocator.  free returns
 * a block obtained from alloc, with the same stream and ctx. */
typedef void *(*h2b_alloc_fn)(size_t bytes, void *hip_stream, void *ctx);
typedef void (*h2b_free_fn)(void *ptr, void *hip_stream, void *ctx);

/* Installs the allocator of all device memory the library takes from now on:
 * operator storage (nearfield, bases, couplings, transposed copies,
 * descriptors), product work vectors, batch and solver work vectors.  With
 * alloc = free = NULL the library uses hipMalloc and hipFree again (the
 * default).  The setting is process-wide.  Every block remembers the
 * allocator it came from and is returned to it (so blocks taken before a
 * change are still freed correctly); before it returns a block the library
 * waits for the device (as hipFree does), so the allocator may hand the block
 * out again at once.  A NULL result of alloc makes the call that needed the
 * memory fail with H2B_ENOMEM, with no handle created and no output written;
 * a block that is not 256-byte aligned is returned and the call fails with
 * H2B_EINVAL.  The Python binding installs torch's caching allocator at
 * import, so the operators' memory shows in torch.cuda.memory_allocated().
 * Errors: H2B_EINVAL if exactly one of alloc and free is NULL. */
h2b_status h2b_set_allocator(h2b_alloc_fn alloc, h2b_free_fn free, void *ctx);

/* Thread-local text of the last error ("" if none). */
const char *h2b_last_error(void);

/* Library version string. */
const char *h2b_version(void);

/* ------------------------------------------------------------------ mesh */

/* Flat triangle mesh (Section 5 uses such meshes of the unit sphere).
 * vx, vy, vz: nv vertex coordinates; t0, t1, t2: nt triangles as 0-based
 * vertex indices, counter-clockwise seen from outside (the outward normal is
 * (v1-v0) x (v2-v0)).  All arrays are host memory and copied.
 * Errors: H2B_EINVAL for nv < 3, nt < 1, an index out of range, a triangle with
 * repeated vertices or zero area, or a non-finite coordinate. */
h2b_status h2b_mesh_create(int64_t nv, const double *vx, const double *vy, const double *vz,
                           int64_t nt, const int32_t *t0, const int32_t *t1, const int32_t *t2,
                           h2b_mesh *out);
h2b_status h2b_mesh_destroy(h2b_mesh mesh);

/* ------------------------------------------------------------------ trees */

/* Cluster tree (Section 2, Definition "Cluster tree") for the triangles (P0,
 * characteristic point = centroid) or the vertices (P1, characteristic point =
 * the vertex): the bounding box of a cluster's characteristic points is split
 * at the midpoint of its longest side (ties: lowest axis; points on the plane
 * go to the first child; if one side would be empty the next-longest axis is
 * tried) while the cluster holds more than leaf_size indices.  Every cluster
 * gets the axis-parallel box B_t of the supports of its basis functions
 * (Section 3).  Host only.
 * Errors: H2B_EINVAL for leaf_size < 1 or a bad space. */
h2b_status h2b_tree_build(h2b_mesh mesh, h2b_space space, int leaf_size, h2b_tree *out);
h2b_status h2b_tree_destroy(h2b_tree tree);

/* Sizes of a tree: number of indices, clusters, leaves and levels. */
h2b_status h2b_tree_info(h2b_tree tree, int64_t *n, int64_t *nclusters, int64_t *nleaves,
                         int32_t *nlevels);

/* Copies of a tree's arrays (host memory, caller-allocated):
 *  perm[n]            original index at each position of the cluster order;
 *  begin/end[nc]      index range perm[begin:end] of each cluster (pre-order,
 *                     first child first);
 *  parent[nc]         parent cluster (-1 for the root);
 *  box[nc*6]          lo_x, lo_y, lo_z, hi_x, hi_y, hi_z of B_t.
 * Any pointer may be NULL. */
h2b_status h2b_tree_arrays(h2b_tree tree, int32_t *perm, int32_t *begin, int32_t *end,
                           int32_t *parent, double *box);

/* Green cross approximation of a tree's cluster bases (Section 4; see
 * h2b_params.gca_tol): the cross approximation of every cluster, bottom-up,
 * on the host only (no device work).  order_m: Gauss points per direction on
 * each face of the auxiliary box (1..6); eps > 0: tolerance relative to the
 * first pivot.  ranks[nclusters] receives k_t per cluster (pre-order ids);
 * pivots, if not NULL, receives the pivot indices (original triangle or
 * vertex indices) cluster after cluster in pivot order, at most
 * sum_t min(|t|, 12 m^2) entries (npivots receives the number written).
 * The operators built with gca_tol use the same construction.
 * Errors: H2B_EINVAL for a NULL tree or ranks, order_m outside 1..6, eps <= 0. */
h2b_status h2b_tree_gca(h2b_tree tree, int order_m, double eps, int32_t *ranks, int32_t *pivots,
                        int64_t *npivots);

/* ----------------------------------------------------------------- blocks */

/* Block tree (Section 2, Definition "Block tree") of rows x cols with the
 * admissibility condition max(diam B_t, diam B_s) <= 2 eta dist(B_t, B_s)
 * (Section 3, eq. (admissibility)): admissible blocks become farfield leaves,
 * pairs of leaf clusters that are not admissible become nearfield leaves.
 * far_disabled != 0 treats no block as admissible (every entry is then a
 * nearfield entry: the dense Galerkin matrix).  Host only.
 * Errors: H2B_EINVAL if the trees belong to different meshes, the rows tree is
 * not P0, or eta <= 0. */
h2b_status h2b_blocks_build(h2b_tree rows, h2b_tree cols, double eta, int far_disabled,
                            h2b_blocks *out);
h2b_status h2b_blocks_destroy(h2b_blocks blocks);

/* Number of farfield and nearfield leaves and nearfield entries. */
h2b_status h2b_blocks_info(h2b_blocks blocks, int64_t *nfar, int64_t *nnear,
                           int64_t *near_entries);

/* Copies of the leaf lists as cluster-id pairs (row, col), in the order of
 * the recursive construction; caller-allocated 2*nfar / 2*nnear int32. */
h2b_status h2b_blocks_lists(h2b_blocks blocks, int32_t *far_pairs, int32_t *near_pairs);

/* --------------------------------------------------------------- assembly */

typedef struct {
    int order_m;            /* Chebyshev points per axis, k = m^3 per cluster; 1..6 */
    int q_near;             /* Gauss points per dimension of the near-field quadrature; 2..16 */
    double recompress_tol;  /* > 0: algebraic recompression of the cluster bases to this
                               relative tolerance (Section 5): orthogonalise the nested bases,
                               weight each cluster by its farfield blocks and its ancestors',
                               truncate, project the couplings; applies to the interpolation and
                               to the gca_tol bases.  Ranks above 64 (order_m 5-6, cross
                               approximation) need an FP64 far field (H2B_ENOTSUP otherwise);
                               0: the bases as built */
    h2b_dtype farfield_dtype; /* storage/arithmetic of bases and coupling matrices */
    int transposed_copy;    /* 1: also store the nearfield and coupling matrices transposed and
                               grouped by column cluster, so that A^T x streams rows like A x
                               (twice that storage); 0: A^T x reads the one copy by columns */
    int symmetric_near;     /* 1: for G on one cluster tree (rows == cols) with leaves of at most 64
                               triangles, also store every pair of nearfield leaves once (N_tt and
                               N_ts, s > t) plus the sparse difference G_ji - G_ij of the touching
                               pairs across leaves; the single-vector products G x and G^T x then
                               read about half the nearfield bytes (0.53x the nearfield storage
                               extra).  With stored FP64 or FP32 couplings (interpolation or
                               gca_tol; not recompute_coupling) of rank at most 256 the coupling
                               matrices are also stored once per pair of clusters (S_ts for s > t;
                               S_st is its transpose to rounding), which halves the coupling bytes
                               of those products (0.5x the coupling storage extra).  Ignored
                               otherwise. */
    double gca_tol;         /* > 0: far field by the Green cross approximation of Section 4
                               instead of interpolation: order_m Gauss points per direction on each
                               face of the auxiliary box omega_t (B_t widened by its largest side),
                               cross approximation of [A C] with full pivoting stopped at gca_tol
                               relative to the first pivot, nested bases V_t by algebraic
                               interpolation and couplings A|_{t_hat x s_hat} from the nearfield
                               quadrature; bases built on the host.  For K the vertex clusters use
                               the normal derivative in y of Green's formula (Section 5).  G must
                               be on one tree (H2B_ENOTSUP otherwise); with recompress_tol > 0 the
                               cross-approximation bases are recompressed (FP64 far field only);
                               0 (default): interpolation */
    int recompute_coupling; /* 1: store no coupling matrices; every product evaluates
                               S_ts = g(xi_t, xi_s) at the interpolation points again (Section 2,
                               eq. (vsw); Section 3), trading their storage (the largest stored
                               object: k^2 values per farfield block) for k_t k_s kernel evaluations
                               per block.  With recompression the projections of the recompressed
                               bases onto the interpolation bases are stored instead (k'_t k values
                               per cluster) and applied once per cluster.  FP64 far field only and
                               not with gca_tol (H2B_ENOTSUP); 0 (default): stored couplings */
} h2b_params;

/* Fills p with the defaults: order_m 4, q_near 4, recompress_tol 0, F64,
 * transposed_copy 1, symmetric_near 1, gca_tol 0, recompute_coupling 0. */
void h2b_params_default(h2b_params *p);

/* Assembles G (kernel H2B_SLP, cols tree P0) or K (H2B_DLP, cols tree P1) on
 * the current HIP device, on hip_stream, and waits for it:
 *  - near field: entries of every nearfield leaf by Sauter-Schwab regularised
 *    quadrature with q_near^4 points per region (Section 5, Table 1);
 *  - far field: m-th order tensor Chebyshev interpolation of g on B_t x B_s
 *    (Section 3): G|ts ~ V_t S_ts W_s^T with (V_t)_{i nu} = int psi_i L_{t,nu},
 *    S_ts = g(xi_{t,nu}, xi_{s,mu}), (W_s)_{j mu} = int psi_j L_{s,mu} for G and
 *    int phi_j dL_{s,mu}/dn for K (derivative of the approximated kernel,
 *    Section 5), with nested transfer matrices (Section 2, eq. (transfer)).
 * Errors: H2B_EINVAL (parameters out of range, kernel/space mismatch),
 * H2B_ENOMEM, H2B_EDEVICE. */
h2b_status h2b_assemble(h2b_blocks blocks, h2b_kernel kernel, const h2b_params *params,
                        void *hip_stream, h2b_op *out);
h2b_status h2b_op_destroy(h2b_op op);

typedef struct {
    int64_t rows, cols;            /* matrix size */
    int64_t nfar, nnear;           /* farfield / nearfield leaves */
    int64_t near_entries;          /* stored nearfield entries */
    int64_t coupling_entries;      /* stored coupling-matrix entries */
    int64_t row_basis_entries;     /* leaf-basis + transfer entries, row tree */
    int64_t col_basis_entries;     /* same, column tree (0 if shared with rows) */
    int64_t bytes_near, bytes_far; /* device bytes of nearfield and farfield data */
    int64_t bytes_vectors;         /* device bytes of the product's work vectors */
    int64_t row_coeffs, col_coeffs; /* cluster coefficients (sum of ranks), row / column tree */
    int32_t max_rank_row, max_rank_col;
    double mean_rank_row, mean_rank_col;
    int64_t bytes_transposed;      /* device bytes of the transposed copies (0 if none) */
    int64_t near_sym_entries;      /* entries of the once-per-pair nearfield (0 if none) */
    int64_t near_sym_columns;      /* its panel columns (one column sum each per product) */
    int64_t near_sym_corrections;  /* touching pairs across leaves (corrections per product) */
    int64_t coupling_evals;        /* kernel evaluations per product (recompute_coupling; else 0) */
    int64_t cpl_sym_entries;       /* entries of the once-per-pair coupling of G (0 if none) */
    int64_t cpl_sym_columns;       /* its panel columns (one column sum each per product) */
} h2b_op_stats;

h2b_status h2b_op_info(h2b_op op, h2b_op_stats *out);

/* ---------------------------------------------------------------- product */

/* y += alpha * op(A) * x for nrhs right-hand sides, A = G or K, op(A) = A
 * (trans = 0) or A^T (trans = 1).  This is the H^2 matrix-vector product
 * (Section 2): forward transformation (leaf bases, then transfer matrices up
 * the column tree), coupling products over the farfield leaves, backward
 * transformation down the row tree, and the nearfield blocks.
 * x: device array of (trans ? rows : cols) x nrhs doubles, column j at x + j*ldx;
 * y: device array of (trans ? cols : rows) x nrhs doubles, column j at y + j*ldy.
 * With nrhs > 1 the right-hand sides are processed in blocks (16, 32 or 64
 * columns, chosen by h2b_op_tune or from nrhs) as small GEMMs that read every
 * stored matrix once per block; the nearfield and coupling blocks of groups up
 * to 64 rows run on matrix cores (MFMA: FP64 nearfield, FP32/FP64 coupling
 * with accumulation in its type, BF16 coupling with FP32 accumulation).  The first call with
 * nrhs > 1 allocates the block work vectors unless h2b_op_tune did.
 * Runs asynchronously on hip_stream: the nearfield runs on a stream of the
 * operator's own that is forked from hip_stream after x is read into the
 * operator's work vector and joined back before y is written, so the call is
 * ordered on hip_stream like a single kernel.  While hip_stream is being
 * captured into a graph, the whole product stays on hip_stream, with the
 * nearfield and the far field as two parallel branches of the graph.  The work vectors belong to the
 * operator: products on one operator must not overlap (same stream, or ordered
 * by the caller).  x and y must not overlap.
 * Errors: H2B_EINVAL (NULL pointers, nrhs < 1 or > 64, ld too small), H2B_EDEVICE. */
h2b_status h2b_matvec(h2b_op op, int trans, double alpha, const double *x, int64_t ldx,
                      double *y, int64_t ldy, int nrhs, void *hip_stream);

/* Size of the static device array that holds the work vectors of
 * h2b_matvec_noalloc (128 MiB on every GPU the library runs on, held until
 * the process ends). */
#define H2B_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): h2b_matvec with
 * every work vector of the product (the permuted input and output, the
 * nearfield output, the cluster coefficients; per block of right-hand sides
 * for nrhs > 1) placed in a static device array of H2B_NOALLOC_SCRATCH_BYTES
 * instead of the operator's own vectors.  The call allocates nothing: no
 * hipMalloc, no installed allocator, no events.  Same arguments, result and
 * asynchronous behaviour as h2b_matvec, except that the nearfield of G is
 * read from its full storage (the once-per-pair form needs the operator's
 * column-sum vector) and no phase timing is recorded.  The work vectors need
 * 3 max(rows, cols) rb doubles plus 2 max(cluster coefficients) rb far-field
 * values (rb = 1 for nrhs = 1, else the block width 16, 32 or 64), each
 * rounded up to 256 bytes; larger requests fail with H2B_EINVAL before any
 * launch.  Every call on a GPU uses that GPU's one array, which keeps the
 * contents of the last call: calls that overlap in time on one GPU (on
 * different streams, or from several threads) race and give wrong results;
 * order them on one stream.  Errors: as h2b_matvec, and H2B_EINVAL for work
 * vectors beyond the array. */
h2b_status h2b_matvec_noalloc(h2b_op op, int trans, double alpha, const double *x, int64_t ldx,
                              double *y, int64_t ldy, int nrhs, void *hip_stream);

/* Batched products over several operators (e.g. meshes of different sizes):
 * captures y_i += alpha_i op_i(A_i) x_i for i < nops into one HIP graph.  The
 * products of different operators are concurrent branches of the graph; each
 * product keeps its phases in sequence inside its branch.
 * The arrays give per-operator arguments as for h2b_matvec; the device
 * vectors are bound at creation and must stay valid while the batch exists.
 * Creation checks every argument first and allocates each operator's work
 * vectors; h2b_batch_launch then replays the graph on hip_stream.
 * The batch keeps no reference to the operators: they must outlive it, and an
 * operator may appear only once per batch and must not run other products
 * while a launch of the batch is in flight.
 * Errors: H2B_EINVAL (bad arguments, repeated operator), H2B_EDEVICE. */
h2b_status h2b_batch_create(int nops, const h2b_op *ops, const int *trans, const double *alpha,
                            const double *const *x, const int64_t *ldx, double *const *y,
                            const int64_t *ldy, const int *nrhs, void *hip_stream, h2b_batch *out);
h2b_status h2b_batch_launch(h2b_batch batch, void *hip_stream);
h2b_status h2b_batch_destroy(h2b_batch batch);

/* Autotuner for products with nrhs (2..64) right-hand sides: times the
 * coupling product of this operator for block widths of 16, 32 and 64
 * right-hand sides (and, for the BF16 far field, two staging depths of panel
 * columns), keeps the fastest for later h2b_matvec calls with nrhs > 1,
 * and allocates the block work vectors (so that later products allocate
 * nothing).  best_us (may be NULL) receives the tuned coupling time in
 * microseconds for nrhs columns.  Synchronises hip_stream.
 * Errors: H2B_EINVAL for nrhs outside 2..64. */
h2b_status h2b_op_tune(h2b_op op, int nrhs, void *hip_stream, double *best_us);

/* Shape derivatives.  Both calls keep the cluster trees, block tree, boxes and
 * Chebyshev points of the operator frozen at the geometry it was assembled
 * for; only the near-field entries and the leaf bases depend on the vertex
 * coordinates.  Operators with recompress_tol > 0 are not supported
 * (H2B_ENOTSUP).
 *
 * h2b_op_set_geometry: new vertex coordinates (host arrays, nv each, same
 * triangles); re-assembles the near field and the leaf bases, synchronises
 * hip_stream.  Errors: H2B_EINVAL for non-finite coordinates or a zero-area
 * triangle.
 *
 * h2b_slp_shape_grad: (gvx, gvy, gvz) += d(x^T G y)/d(vertex coordinates) for
 * the H^2 approximation of G (Section 1, eq. (slp)): the adjoint of the
 * near-field quadrature (every stored entry weighted by x_i y_j) plus the
 * derivative of the leaf-basis integrals weighted by the leaf coefficients of
 * the two partial products S V^T y and S V^T x (the far field is symmetric,
 * S_st = S_ts^T).  x, y: device arrays of nt doubles (triangle order);
 * gvx, gvy, gvz: device arrays of nv doubles (vertex order), accumulated
 * with atomics.  Runs asynchronously on hip_stream.
 * Errors: H2B_EINVAL if the operator is not G or a pointer is NULL. */
h2b_status h2b_op_set_geometry(h2b_op op, const double *vx, const double *vy, const double *vz,
                               void *hip_stream);
h2b_status h2b_slp_shape_grad(h2b_op G, const double *x, const double *y, double *gvx, double *gvy,
                              double *gvz, void *hip_stream);

/* The discrete single-layer bilinear form b = x^T G y (Section 1, eq. (slp),
 * with the H^2 approximation of G): gy = G y (overwritten) and
 * out[0] = x^T gy, an FP64 inner product reduced in a fixed order (the same
 * bits for the same input on the same device).  x, y, gy: device arrays of nt
 * doubles (triangle order); out: one device double.  This is the forward
 * value of the shape-differentiable form whose derivative
 * h2b_slp_shape_grad gives; gy is kept for the derivative in x.  Uses the
 * operator's work vectors (no overlap with other calls on G).  Runs
 * asynchronously on hip_stream.
 * Errors: H2B_EINVAL if G is not the single-layer operator, for a NULL
 * pointer, gy overlapping x or y, or out overlapping x or gy. */
h2b_status h2b_slp_bilinear(h2b_op G, const double *x, const double *y, double *gy, double *out,
                            void *hip_stream);

/* Per-phase timing of the products on an operator, measured with HIP events on
 * the streams the phases run on.  A product runs its nearfield on a stream of
 * the operator's own, forked from hip_stream after the gather and joined
 * before the scatter, so that it overlaps the far field (forward
 * transformation, coupling, backward transformation) on hip_stream.
 * h2b_op_set_timing(op, 1) starts recording (one event set per product,
 * created on the host as needed); h2b_op_phase_times waits for the last
 * recorded product and returns the mean milliseconds per product of
 * phases[0..6] = gather, forward transformation, coupling, backward
 * transformation, nearfield, scatter, whole product, then restarts the
 * average.  The coupling phase contains one kernel launch, the nearfield
 * phase one (two with the once-per-pair storage of G: the panel pass and the
 * reduction of its column sums).  Errors: H2B_ESTATE if nothing was recorded. */
h2b_status h2b_op_set_timing(h2b_op op, int enable);
h2b_status h2b_op_phase_times(h2b_op op, double phases_ms[7]);

/* Overlap of the nearfield with the far field (default 1).  With 0 every
 * phase of the products of op runs on the caller's stream, one kernel after
 * the other (for callers that schedule their own concurrent work, and for
 * timing each kernel alone).  The result is the same either way.
 * Errors: H2B_EINVAL if op is NULL. */
h2b_status h2b_op_set_overlap(h2b_op op, int enable);

/* ------------------------------------------------ Dirichlet-to-Neumann solve */

/* Mixed mass matrix M (Section 1): m_ij = int psi_i phi_j for the triangle
 * indicator psi_i and the hat function phi_j of vertex j, i.e. |tau_i| / 3
 * when j is a corner of tau_i and 0 otherwise.  trans = 0: y += alpha M x
 * with x on the vertices (nv doubles, vertex order) and y on the triangles
 * (nt doubles, triangle order); trans = 1: y += alpha M^T x (x on the
 * triangles, y on the vertices).  op is any operator assembled on the mesh
 * and supplies its device geometry (the current one after
 * h2b_op_set_geometry).  x and y are device arrays that must not overlap.
 * Runs asynchronously on hip_stream.  Errors: H2B_EINVAL for a NULL pointer
 * or overlapping x and y.
 *
 * With the double-layer operator K this gives the right-hand side
 * (M/2 + K) u of the Dirichlet-to-Neumann system G t = (M/2 + K) u
 * (Section 1, eq. (matrix_dtn)) from the Dirichlet coefficients u. */
h2b_status h2b_mass_matvec(h2b_op op, int trans, double alpha, const double *x, double *y,
                           void *hip_stream);

/* Hypersingular matrix W (Section 1, eq. for w_ij), set up through its
 * representation by the single-layer operator that the paper uses: for the
 * hat functions on flat triangles w_ij is the sum over triangle pairs of
 * <curl phi_i on tau, curl phi_j on tau'> times the single-layer entry
 * g_{tau tau'}, i.e. W = sum_d C_d^T G C_d, where the surface curl
 * n x grad phi_j is constant on each triangle (corners (a, b, c)
 * counter-clockwise: curl phi_a = (x_b - x_c) / (2 |tau|), cyclically).
 * y += alpha W x with x, y device arrays of nv doubles (vertex order).  G is
 * the H^2 single-layer operator of the mesh (any precision settings); one
 * call is two small curl kernels around three products of G.  The first call allocates 6 nt doubles of work vectors
 * on the operator.  W annihilates constants.  Runs asynchronously on
 * hip_stream.  Errors: H2B_EINVAL if G is not the single-layer operator, for
 * NULL or overlapping x and y. */
h2b_status h2b_hypersingular_matvec(h2b_op G, double alpha, const double *x, double *y, void *hip_stream);

/* Conjugate gradients for A x = b with the H^2 product of a square operator
 * (meant for the symmetric positive definite single-layer matrix G of eq.
 * (matrix_dtn); the Krylov solver of the experiments in Section 5).
 *
 * Iteration (Hestenes-Stiefel): q = A p, alpha = rho / p^T q,
 * x += alpha p, r -= alpha q, rho' = r^T r, p = r + (rho'/rho) p.  Inner
 * products are double precision, reduced in a fixed order (the same result
 * for the same input on the same device).  Stops at the first iterate with
 * ||r_k||_2 <= tol ||b||_2 (r_k the updated residual; absolute when b = 0),
 * after max_iter iterations, or on breakdown (p^T q not positive or not
 * finite).  Every scalar of the iteration stays on the device: the host
 * queues check_every iterations at a time (captured once into a HIP graph,
 * in which each product runs its nearfield and far field as parallel
 * branches, and replayed when use_graph = 1) and then reads the state.  The iterations
 * queued after the stopping one change nothing (x, r and the count are
 * frozen), so the result does not depend on check_every or use_graph.  The
 * products of A inside the iteration run with A's precision settings (a
 * lower-precision far field makes CG solve the perturbed system).
 *
 * With form = H2B_FORM_HYPERSINGULAR the operator is instead the
 * hypersingular matrix W built from the single-layer operator A = G (see
 * h2b_hypersingular_matvec), for the Neumann-to-Dirichlet system
 * W u = (M^T/2 - K^T) t of eq. (matrix_ntd).  W is only semi-definite
 * (constants span its null space) and such a right-hand side is orthogonal
 * to the constants only up to quadrature error, so b is first replaced by
 * b - c w1 with w1_j = int phi_j and c = 1^T b / 1^T w1 (the consistent
 * system of the solve bordered by w1), CG runs on that (the residuals and
 * tol refer to it), and the solution is returned with int u_h = w1^T x = 0.
 *
 * b: device array of n doubles; x: device array of n doubles, the initial
 * guess on entry (ignored and set to 0 when zero_guess = 1) and the last
 * iterate on return; n = rows = columns of A (the number of vertices for the
 * hypersingular form).  history: NULL, or a host array
 * of max_iter + 1 doubles receiving ||r_k|| / ||b|| for k = 0..iterations.
 * Work vectors (3 n doubles, one more with the preconditioner and two more
 * for the hypersingular form, plus small state) are allocated per call.  The
 * call synchronises hip_stream and returns when the solve has ended.
 * precond = H2B_PRECOND_BLOCK_JACOBI runs preconditioned CG (rho = r^T z,
 * z = P r) with P the block-diagonal matrix of the inverses of the symmetric
 * parts of the diagonal nearfield blocks N_tt of the leaves (G on one tree,
 * leaves of at most 64; product form only).  The inverses are computed on
 * the device by the first such solve (sum of |t|^2 doubles, kept by the
 * operator); applying P reads them once per iteration.  The stopping test
 * and the residuals stay on ||r||.  This is a simpler stand-in for the
 * paper's preconditioner.  precond = H2B_PRECOND_HCHOL runs preconditioned CG
 * with z = (L L^T)^{-1} r from the factor params.hchol (see
 * h2b_hchol_build; the paper's preconditioner), whose size must be n; product
 * form only.
 *
 * Errors: H2B_EINVAL for a non-square operator (not the single-layer
 * operator for the hypersingular form), an unknown form or preconditioner,
 * NULL or overlapping b and x, tol < 0 or not finite, max_iter < 0,
 * check_every < 1, H2B_PRECOND_HCHOL with a NULL factor or one of another
 * size; H2B_ENOTSUP for the block-Jacobi preconditioner on other operators,
 * larger leaves, and for either preconditioner with the hypersingular
 * form. */
typedef enum { H2B_FORM_PRODUCT = 0, H2B_FORM_HYPERSINGULAR = 1 } h2b_cg_form;
typedef enum { H2B_PRECOND_NONE = 0, H2B_PRECOND_BLOCK_JACOBI = 1, H2B_PRECOND_HCHOL = 2 } h2b_cg_precond;

/* ---------------------------------------------- H-Cholesky preconditioner
 *
 * The paper preconditions its conjugate gradient solves by coarsening the
 * compressed matrix to a relative accuracy eps_prc and factorising it,
 * G ~ L L^T, in H-matrix arithmetic (Section 1; the eps_prc column of the
 * parameter table of Section 5).  Here:
 *  - the lower triangle of G becomes an H-matrix on its cluster and block
 *    trees: a farfield block V_t S_ts V_s^T the low-rank product U V^T with
 *    U = V_t S_ts and V = V_s (the parent bases made explicit through the
 *    transfer matrices of Section 2, eq. (transfer)), a nearfield block a
 *    dense array;
 *  - coarsening: every low-rank block is truncated to the singular values
 *    above eps times its largest, every off-diagonal dense block made
 *    low-rank where that stores fewer values, and, from the leaves up, every
 *    off-diagonal subdivided block whose parts are all leaves replaced by one
 *    truncated low-rank block where that stores fewer values;
 *  - H-Cholesky: L11 = chol(G11), L21 = G21 L11^{-T}, L22 = chol(G22 - L21 L21^T)
 *    recursively over the diagonal blocks, every product of blocks formed in
 *    low-rank or dense arithmetic and every low-rank result truncated to eps.
 * Setup runs on the host (the values of G are copied from the device once).
 * Applying z = (L L^T)^{-1} r runs on the device: forward and backward
 * substitution over the block recursion, flattened into a list of steps of
 * independent tasks (the inverse of a dense diagonal factor, the
 * coefficients V^T y of the low-rank blocks of an update, the rows of a leaf
 * cluster changed by an update) run by one workgroup, since the chain of
 * diagonal leaves is sequential. */
typedef struct h2b_hchol_s *h2b_hchol;

typedef struct {
    int64_t n;                      /* rows */
    double eps;                     /* truncation accuracy */
    int64_t coarse_entries;         /* stored doubles after coarsening */
    int64_t dense_entries;          /* stored doubles of the factor in dense blocks */
    int64_t rk_entries;             /* ... and in low-rank blocks */
    int64_t dense_blocks, rk_blocks;
    int max_rank;                   /* largest rank of a block of the factor */
    int64_t coarsened_blocks;       /* subdivided blocks replaced by one low-rank block */
    int64_t converted_blocks;       /* dense blocks replaced by low-rank ones */
    int64_t steps, tasks;           /* substitution program: steps and tasks of both sweeps (0 before
                                       the first device use) */
    double convert_s, coarsen_s, factor_s, upload_s;  /* host wall time of the setup stages */
} h2b_hchol_info;

/* Builds the preconditioner of the single-layer operator G (FP64 far field,
 * stored couplings, one cluster tree for rows and columns) to accuracy
 * eps >= 0 (0: exact up to rounding, dense storage) and uploads its
 * substitution program.  Synchronises hip_stream.  Errors: H2B_EINVAL for a
 * NULL or non-single-layer G, eps < 0 or not finite; H2B_ENOTSUP for other
 * far-field settings, dense diagonal leaves above 256 rows, or a pivot that
 * is not positive (the coarsened matrix is not positive definite at this eps:
 * use a smaller one). */
h2b_status h2b_hchol_build(h2b_op G, double eps, h2b_hchol *out, void *hip_stream);

/* The same from a dense symmetric matrix A (n x n, row-major, host memory,
 * the caller's numbering of the blocks' tree; n = tree size) on the blocks of
 * one P0 tree: nearfield leaves copied, farfield leaves truncated to eps by
 * a singular value decomposition.  Host only (no device use until
 * h2b_hchol_apply).  Errors: H2B_EINVAL for NULL arguments, blocks on two
 * trees, eps < 0; H2B_ENOTSUP as above. */
h2b_status h2b_hchol_from_dense(h2b_blocks blocks, const double *A, double eps, h2b_hchol *out);

/* z = (L L^T)^{-1} r on the host (r, z: host arrays of n doubles, caller's
 * numbering; may be the same array). */
h2b_status h2b_hchol_solve_host(h2b_hchol P, const double *r, double *z);

/* z = (L L^T)^{-1} r on the device (r, z: device arrays of n doubles, caller's
 * numbering, not overlapping), asynchronous on hip_stream.  The first call
 * uploads the program if the handle came from h2b_hchol_from_dense.  Uses
 * the handle's work vectors: calls on one handle must not overlap. */
h2b_status h2b_hchol_apply(h2b_hchol P, const double *r, double *z, void *hip_stream);

h2b_status h2b_hchol_get_info(h2b_hchol P, h2b_hchol_info *info);
h2b_status h2b_hchol_destroy(h2b_hchol P);

typedef struct {
    double tol;        /* relative residual to reach (default 1e-8) */
    int max_iter;      /* iteration limit (default 1000) */
    int check_every;   /* iterations queued between two reads of the state (default 8) */
    int use_graph;     /* 1: replay a HIP graph of check_every iterations (default 1) */
    int zero_guess;    /* 1: start from x = 0 without the initial product (default 1) */
    int form;          /* h2b_cg_form: the operator's product (default) or W built from G */
    int precond;       /* h2b_cg_precond: none (default), block Jacobi or H-Cholesky, see below */
    h2b_hchol hchol;   /* the factor for H2B_PRECOND_HCHOL (NULL otherwise; default NULL) */
} h2b_cg_params;

typedef enum { H2B_CG_CONVERGED = 1, H2B_CG_BREAKDOWN = 2, H2B_CG_MAXITER = 3 } h2b_cg_status;

typedef struct {
    int iterations;       /* iterations done */
    int status;           /* h2b_cg_status */
    double rel_residual;  /* ||r_k|| / ||b|| of the last iterate */
    double solve_ms;      /* wall time of the call, including the graph build */
} h2b_cg_result;

void h2b_cg_params_default(h2b_cg_params *p);
h2b_status h2b_cg_solve(h2b_op A, const double *b, double *x, const h2b_cg_params *params,
                        h2b_cg_result *result, double *history, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* H2BEM_H */
