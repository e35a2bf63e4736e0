// Batched products over several operators (meshes of different sizes)
// captured once into a hipGraph.  Products that share one program (same
// far-field type, direction and number of right-hand sides) are merged step by
// step (batch_merged.hip).  Otherwise each operator's product starts
// a new root of the graph (the stream's capture dependencies are cleared
// before it), so the products of different meshes are independent branches.
// Inside the batch each product keeps its phases in sequence: splitting every
// product further into nearfield and far-field branches made the graph of 16
// meshes (2,048 to 32,768 triangles) three times slower on the MI355X (3.3 ms
// against 1.1 ms), while a product captured alone gains from the split.  The
// capture ends after every branch; one graph launch runs the whole batch.
#include <hip/hip_runtime.h>

#include <set>
#include <utility>
#include <vector>

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
    }
    // the caller's stream may be the null stream, which cannot be captured:
    // capture on a private stream and launch the graph on the caller's
    // stream later
    auto b = std::make_unique<Batch>();
    b->streams.resize(1, nullptr);
    hip_check(hipStreamCreateWithFlags(&b->streams[0], hipStreamNonBlocking), "stream create");
    hipStream_t cap = b->streams[0];
    // products that share one program run merged: one launch per step for the
    // whole batch, with work vectors of the batch's own
    b->merged = merged_create(nops, ops, trans, alpha, x, ldx, y, ldy, nrhs, st);
    if (b->merged) {
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
            merged_capture(*b->merged, cap);
        } catch (...) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cap, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(cap, &b->graph), "end capture");
        hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
        return b;
    }
    // the graph keeps the addresses of the operators' work vectors: block
    // vectors are reserved at the widest block so that nothing reallocates
    // them while the batch exists (a later h2b_op_tune or wider product)
    for (int i = 0; i < nops; ++i)
        if (nrhs[i] > 1) reserve_block_buffers(*ops[i]);
    // the products stay sequential inside the capture (overlap off), restored
    // on every exit
    struct OverlapOff {
        std::vector<std::pair<Op *, bool>> saved;
        ~OverlapOff()
        {
            for (auto &o : saved) o.first->overlap = o.second;
        }
    } guard;
    for (int i = 0; i < nops; ++i) {
        guard.saved.push_back({ops[i], ops[i]->overlap});
        ops[i]->overlap = false;
    }
    hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
    try {
        std::vector<hipGraphNode_t> ends;
        for (int i = 0; i < nops; ++i) {
            if (i > 0) set_capture_tail(cap, {});
            matvec(*ops[i], trans[i], alpha[i], x[i], ldx[i], y[i], ldy[i], nrhs[i], cap);
            const std::vector<hipGraphNode_t> e = capture_tail(cap);
            ends.insert(ends.end(), e.begin(), e.end());
        }
        set_capture_tail(cap, ends);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hip_check(hipStreamEndCapture(cap, &b->graph), "end capture");
    hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate");
    return b;
}

void batch_launch(Batch &b, hipStream_t st) { hip_check(hipGraphLaunch(b.exec, st), "graph launch"); }

}  // namespace h2b
