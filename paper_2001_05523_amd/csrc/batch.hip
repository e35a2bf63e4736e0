// Batched products over several operators (meshes of different sizes)
// captured once into a hipGraph: every operator gets its own stream forked
// from the caller's stream during capture, so the products of different
// meshes are independent graph branches that run concurrently; one graph
// launch runs the whole batch.
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
    // capture on a private origin stream (streams[nops]) and launch the graph
    // on the caller's stream later
    (void)st;
    auto b = std::make_unique<Batch>();
    b->streams.resize(nops + 1, nullptr);
    b->events.resize(nops + 1, nullptr);
    for (auto &s : b->streams) hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream create");
    for (auto &e : b->events) hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create");
    hipStream_t origin = b->streams[nops];
    hip_check(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
        hip_check(hipEventRecord(b->events[nops], origin), "fork");
        for (int i = 0; i < nops; ++i) {
            hip_check(hipStreamWaitEvent(b->streams[i], b->events[nops], 0), "fork");
            matvec(*ops[i], trans[i], alpha[i], x[i], ldx[i], y[i], ldy[i], nrhs[i], b->streams[i]);
            hip_check(hipEventRecord(b->events[i], b->streams[i]), "join");
            hip_check(hipStreamWaitEvent(origin, b->events[i], 0), "join");
        }
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(origin, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hip_check(hipStreamEndCapture(origin, &b->graph), "end capture");
    hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    return b;
}

void batch_launch(Batch &b, hipStream_t st) { hip_check(hipGraphLaunch(b.exec, st), "graph launch"); }

}  // namespace h2b
