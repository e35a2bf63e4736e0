// Device-side inputs and kernel launchers of the H^2 library.
#pragma once

#include <hip/hip_runtime.h>

#include "panels.hpp"

namespace h2b {

using bf16_t = __bf16;     // storage type of the BF16 coupling matrices

constexpr int QMAX = 16;   // largest Gauss order per dimension
constexpr int MMAX = 6;    // largest Chebyshev order per axis

// Mesh in device memory (structure of arrays).
struct GeoDev {
    const double *vx, *vy, *vz;
    const int32_t *t0, *t1, *t2;
    const double *nx, *ny, *nz;
    const int64_t *vt_ptr;
    const int32_t *vt_idx;
};

// Gauss-Legendre rule on [0,1], passed by value to the kernels.
struct QuadDev {
    int q;
    double t[QMAX];
    double w[QMAX];
};

// ------------------------------------------------------------- assembly

// Nearfield entries of every group of rp (one workgroup per group).
// kernel H2B_SLP: vals = G_ij; H2B_DLP: vals = K_ij (column j = vertex).
void launch_near_assemble(h2b_kernel kernel, const RowPanels &rp, const int32_t *rperm,
                          const int32_t *cperm, const GeoDev &geo, const QuadDev &quad,
                          double *vals, hipStream_t st);

// Double-layer nearfield with every triangle pair integrated once per row:
// lst[lptr[g] .. lptr[g + 1]) is the sorted list of the triangles around the
// column vertices of group g.
void launch_near_assemble_dlp(const RowPanels &rp, const int64_t *lptr, const int32_t *lst, const int32_t *rperm,
                              const int32_t *cperm, const GeoDev &geo, const QuadDev &quad, double *vals,
                              hipStream_t st);

// Leaf bases stored as V_t^T (k x |t| per leaf group of rp).
// space P0: (V_t)_{i nu} = int_{tau_i} L_{t,nu};
// dlp_cols (space P1): (W_t)_{j nu} = sum_{tau around j} int_tau phi_j dL_{t,nu}/dn_tau.
template <typename T>
void launch_leaf_basis(bool dlp_cols, const RowPanels &rp, const int32_t *perm,
                       const double *axes, int m, const GeoDev &geo, const QuadDev &quad,
                       T *vals, hipStream_t st);

// Transfer panels [E_c0^T | E_c1^T], (E_c)_{mu nu} = L_{t,nu}(xi_{c,mu}).
template <typename T>
void launch_transfer(const RowPanels &rp, const double *axes, int m, T *vals, hipStream_t st);

// Coupling panels, S_ts[nu, mu] = g(xi_{t,nu}, xi_{s,mu}).
template <typename T>
void launch_coupling(const RowPanels &rp, const double *raxes, const double *caxes, int m, T *vals,
                     hipStream_t st);

// Shape derivative of x^T G y: near-field entries (every stored (i, j) with
// weight x_i y_j) and leaf bases (coefficients x_i a_t(y) + y_i a_t(x)), added
// into the vertex gradient arrays gx, gy, gz.
void launch_near_grad(const RowPanels &rp, const int32_t *perm, const GeoDev &geo, const QuadDev &quad,
                      const double *xp, const double *yp, double *gx, double *gy, double *gz, hipStream_t st);
template <typename F>
void launch_leaf_grad(const RowPanels &leaf, const int32_t *perm, const double *axes, int m, const GeoDev &geo,
                      const QuadDev &quad, const F *ax, const F *ay, const double *xp, const double *yp,
                      double *gx, double *gy, double *gz, hipStream_t st);

// --------------------------------------------------------------- product

// Step of the product a panel launch belongs to; each gets its own kernel
// instance so that profiles tell them apart.
enum class Role { Leaf, Transfer, Coupling, Near };

// y[out_begin + r] (=|+=) sum_c vals[...] x[...] for groups [g0, g1).
template <typename VT, typename XT, typename YT>
void launch_rowpanel(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y,
                     bool accumulate, hipStream_t st, Role role);

// y[out_begin + j] (+)= sum over blocks of the transposed product, groups [g0, g1)
// (overwrite only for the leaf and transfer roles).
template <typename VT, typename XT, typename YT>
void launch_colpanel(const ColPanels &cp, int g0, int g1, const VT *vals, const XT *x, YT *y,
                     hipStream_t st, Role role, bool accumulate = true);

// out = per-group transpose of the panels of rp (same offsets).
template <typename T> void launch_transpose_panels(const RowPanels &rp, const T *in, T *out, hipStream_t st);

// Many right-hand sides, vectors stored row-major per block of rb columns
// (entry (i, r) at i * rb + r), rb in {16, 32, 64}.
template <typename VT, typename XT, typename YT>
void launch_rowpanel_mrhs(const RowPanels &rp, int g0, int g1, int rb, const VT *vals, const XT *x, YT *y,
                          bool accumulate, hipStream_t st, Role role);
// Coupling on matrix cores: FP32 or BF16 panels, FP32 vectors and accumulation,
// kc = input columns staged per step (32 or 64).
template <typename VT>
void launch_rowpanel_mrhs_mfma(const RowPanels &rp, int g0, int g1, int rb, int kc, const VT *vals,
                               const float *x, float *y, bool accumulate, hipStream_t st);
// Y (+)= P X for every group (at most 64 rows) on matrix cores, FP32 or FP64,
// columns split over the four waves of a group, operands read directly.
template <typename T>
void launch_panel_mfma(const RowPanels &rp, int g0, int g1, int rb, const T *vals, const T *x, T *y,
                       bool accumulate, hipStream_t st);
template <typename VT, typename XT, typename YT>
void launch_colpanel_mrhs(const ColPanels &cp, int g0, int g1, int rb, const VT *vals, const XT *x, YT *y,
                          bool accumulate, hipStream_t st, Role role);
void launch_gather_mrhs(const int32_t *perm, int64_t n, int nb, int rb, const double *x, int64_t ldx,
                        double *xp, hipStream_t st);
// y[perm[k] + r*ldy] += alpha * (yp[k*rb + r] + yp2[k*rb + r]), r < nb; yp2 may be NULL
void launch_scatter_mrhs(const int32_t *perm, int64_t n, int nb, int rb, double alpha, const double *yp,
                         const double *yp2, double *y, int64_t ldy, hipStream_t st);

// xp[k + c*n] = x[perm[k] + c*ldx]
void launch_gather(const int32_t *perm, int64_t n, int nrhs, const double *x, int64_t ldx,
                   double *xp, hipStream_t st);
// y[perm[k] + c*ldy] += alpha * (yp[k + c*n] + yp2[k + c*n]); yp2 may be NULL
void launch_scatter_add(const int32_t *perm, int64_t n, int nrhs, double alpha, const double *yp,
                        const double *yp2, double *y, int64_t ldy, hipStream_t st);
// y[segment entry of column c] += sum_i P[i][c] * x[out_begin + i] for every
// group P of rp in [g0, g1) (leaf and transfer roles; outputs of distinct
// groups must be disjoint).
template <typename VT, typename XT, typename YT>
void launch_rowpanelT(const RowPanels &rp, int g0, int g1, const VT *vals, const XT *x, YT *y, hipStream_t st,
                      Role role);
// Transposed copy of the values `in` of the row panels that cp describes, as
// the row panels `out` built by regroup_transposed(cp, out).
template <typename T>
void launch_regroup_transpose(const ColPanels &cp, const RowPanels &out, const T *in, T *o, hipStream_t st);
template <typename T> void launch_fill_zero(T *p, int64_t n, hipStream_t st);

}  // namespace h2b
