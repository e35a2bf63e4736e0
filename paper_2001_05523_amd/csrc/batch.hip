// Batched products over several operators (meshes of different sizes) built
// once into a hipGraph: the products of different meshes are independent
// branches of the graph, and inside each single-vector product the nearfield
// and the far field are two more parallel branches (prepare -> {nearfield,
// far field} -> scatter).  Every piece is captured alone on one private
// stream and added as a child-graph node, so no capture spans two streams.
// One graph launch runs the whole batch.
#include <hip/hip_runtime.h>

#include <set>

#include "op.hpp"

namespace h2b {

Batch::~Batch()
{
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (auto e : events) (void)hipEventDestroy(e);
    for (auto s : streams) (void)hipStreamDestroy(s);
}

std::unique_ptr<Batch> batch_create(int nops, Op *const *ops, const int *trans, const double *alpha,
                                    const double *const *x, const int64_t *ldx, double *const *y,
                                    const int64_t *ldy, const int *nrhs, hipStream_t st)
{
    if (nops < 1) fail(H2B_EINVAL, "nops must be >= 1");
    if (!ops || !trans || !alpha || !x || !ldx || !y || !ldy || !nrhs) fail(H2B_EINVAL, "NULL array");
    std::set<Op *> seen;
    for (int i = 0; i < nops; ++i) {
        if (!ops[i]) fail(H2B_EINVAL, "NULL operator");
        if (!seen.insert(ops[i]).second)
            fail(H2B_EINVAL, "an operator appears twice (its work vectors would be shared)");
        // argument checks and block buffers happen before the capture
        check_product_args(*ops[i], trans[i], x[i], ldx[i], y[i], ldy[i], nrhs[i]);
        prepare_product(*ops[i], nrhs[i]);
    }
    // the caller's stream may be the null stream, which cannot be captured:
    // capture the pieces on a private stream and launch the graph on the
    // caller's stream later
    (void)st;
    auto b = std::make_unique<Batch>();
    b->streams.resize(1, nullptr);
    hip_check(hipStreamCreateWithFlags(&b->streams[0], hipStreamNonBlocking), "stream create");
    hipStream_t cap = b->streams[0];
    hip_check(hipGraphCreate(&b->graph, 0), "graph create");
    for (int i = 0; i < nops; ++i) {
        if (nrhs[i] == 1)
            add_product_nodes(*ops[i], trans[i], alpha[i], x[i], y[i], b->graph, {}, cap);
        else
            add_captured(b->graph, {}, cap,
                         [&] { matvec(*ops[i], trans[i], alpha[i], x[i], ldx[i], y[i], ldy[i], nrhs[i], cap); });
    }
    hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    return b;
}

void batch_launch(Batch &b, hipStream_t st) { hip_check(hipGraphLaunch(b.exec, st), "graph launch"); }

}  // namespace h2b
