// Green cross approximation (GCA, Section 4) of G and K on the device: the
// bases built on the host (gca_host.cpp) are uploaded, and the coupling
// entries A|_{t_hat x s_hat} come from the nearfield quadrature kernel over
// panels whose rows and columns are pivot triangles (and pivot vertices for
// K's columns).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "linalg.hpp"
#include "op.hpp"

namespace h2b {

namespace {

template <typename TO> __global__ void k_convert(const double *__restrict__ in, TO *__restrict__ out, int64_t n)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (TO)in[e];
}

}  // namespace

namespace {

void set_gca_basis(Basis &B, const GcaBases &G, h2b_dtype dt, hipStream_t st)
{
    const Tree &T = *B.tree;
    // leaf panels hold V_t^T (k_t x |t|), transfer panels [E_1^T | E_2^T]
    std::vector<double> leaf(std::max<int64_t>(B.leaf.total, 1)), tr(std::max<int64_t>(B.trans.total, 1));
    for (int g = 0; g < B.leaf.ngroups(); ++g) {
        const int c = B.leaf.group_tag[g], n = T.size(c), k = G.rank[c];
        for (int nu = 0; nu < k; ++nu)
            for (int i = 0; i < n; ++i) leaf[B.leaf.val_off[g] + (int64_t)nu * n + i] = G.V[c][(size_t)i * k + nu];
    }
    for (int g = 0; g < B.trans.ngroups(); ++g) {
        const int c = B.trans.group_tag[g], k = G.rank[c];
        const int n = G.rank[T.child0[c]] + G.rank[T.child1[c]];
        for (int nu = 0; nu < k; ++nu)
            for (int mu = 0; mu < n; ++mu) tr[B.trans.val_off[g] + (int64_t)nu * n + mu] = G.V[c][(size_t)mu * k + nu];
    }
    auto up = [&](const std::vector<double> &v, DevMem &mem) {
        if (dt == H2B_F64) {
            mem.alloc(v.size() * sizeof(double));
            hip_check(hipMemcpyAsync(mem.p, v.data(), v.size() * sizeof(double), hipMemcpyHostToDevice, st),
                      "upload");
        } else {
            std::vector<float> f(v.begin(), v.end());
            mem.alloc(f.size() * sizeof(float));
            hip_check(hipMemcpyAsync(mem.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice, st),
                      "upload");
        }
        hip_check(hipStreamSynchronize(st), "upload");
    };
    up(leaf, B.leaf_vals);
    up(tr, B.trans_vals);
    transpose_basis_values(B, dt, st);
}

// Original index of the pivot at every coefficient position of a basis.
void upload_pivots(const Basis &B, const GcaBases &G, DevMem &mem, hipStream_t st)
{
    std::vector<int32_t> h(std::max<int64_t>(B.hat_total, 1), 0);
    for (int64_t c = 0; c < B.tree->nclusters(); ++c)
        for (int i = 0; i < G.rank[c]; ++i) h[B.hat_off[c] + i] = G.hat[c][i];
    mem.alloc(sizeof(int32_t) * h.size());
    hip_check(hipMemcpyAsync(mem.p, h.data(), sizeof(int32_t) * h.size(), hipMemcpyHostToDevice, st), "upload");
    hip_check(hipStreamSynchronize(st), "upload");
}

}  // namespace

void set_gca_values(Op &op, const GcaBases &Gr, const GcaBases &Gc, hipStream_t st)
{
    const h2b_dtype dt = op.params.farfield_dtype;
    set_gca_basis(*op.rowb, Gr, dt, st);
    if (op.colb != op.rowb) set_gca_basis(*op.colb, Gc, dt, st);
    DevMem rh, ch;
    upload_pivots(*op.rowb, Gr, rh, st);
    if (op.colb != op.rowb) upload_pivots(*op.colb, Gc, ch, st);
    const int32_t *rperm = rh.as<int32_t>(), *cperm = op.colb != op.rowb ? ch.as<int32_t>() : rperm;
    // couplings: entries A_{i j} for the pivots i of t_hat and j of s_hat
    const int64_t n = std::max<int64_t>(op.cpl.total, 1);
    DevMem s64;
    double *dst = nullptr;
    if (dt == H2B_F64) {
        op.cpl_vals.alloc(sizeof(double) * n);
        dst = op.cpl_vals.as<double>();
    } else {
        s64.alloc(sizeof(double) * n);
        dst = s64.as<double>();
    }
    launch_near_assemble(op.kernel, op.cpl, rperm, cperm, op.geo, make_quad(op.params.q_near), dst, st);
    if (dt != H2B_F64) {
        op.cpl_vals.alloc(coupling_size(dt) * n);
        const int nb = (int)std::min<int64_t>((n + 255) / 256, 65536);
        if (dt == H2B_F32)
            hipLaunchKernelGGL(k_convert<float>, dim3(nb), dim3(256), 0, st, dst, op.cpl_vals.as<float>(), n);
        else
            hipLaunchKernelGGL(k_convert<bf16_t>, dim3(nb), dim3(256), 0, st, dst, op.cpl_vals.as<bf16_t>(), n);
        hip_check(hipGetLastError(), "convert launch");
    }
    hip_check(hipStreamSynchronize(st), "gca couplings");
}

}  // namespace h2b
