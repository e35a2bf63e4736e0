// The H-Cholesky preconditioner: factor on the host, substitutions on the
// device (hchol.hip, hmatrix.cpp).
#pragma once

#include <chrono>
#include <memory>

#include "hmatrix.hpp"
#include "op.hpp"

namespace h2b {

struct HChol {
    std::unique_ptr<HMatrix> H;
    HProgram prog_host;
    double eps = 0.0;
    HStats coarse, factor;  // storage after coarsening and of the factor
    double convert_s = 0.0, coarsen_s = 0.0, factor_s = 0.0, upload_s = 0.0;
    // device program
    bool uploaded = false;
    int64_t n = 0, ntasks = 0, device_values = 0;
    int nsteps = 0, fw_steps = 0;
    DevMem vals, coef, y, prog;
    const int32_t *d_step = nullptr, *d_tasks = nullptr, *d_items = nullptr, *d_perm = nullptr;
};

// The lower triangle of the single-layer operator G as an H-matrix (far
// blocks U V^T with U = V_t S_ts, V = V_s; near blocks copied).
std::unique_ptr<HMatrix> hmatrix_from_op(const Op &op, double eps, hipStream_t st);
// Coarsening and factorisation of P.H to accuracy eps.
void hchol_factor(HChol &P, double eps);
// The substitution program of the factor (once).
void hchol_flatten(HChol &P);
// The program and its values on the device (once).
void hchol_upload(HChol &P, hipStream_t st);
// z = (L L^T)^{-1} r, r and z device vectors in the caller's numbering.
void hchol_apply(HChol &P, const double *r, double *z, hipStream_t st);

}  // namespace h2b

struct h2b_hchol_s {
    std::unique_ptr<h2b::HChol> p;
};
