// Batched products and tile tuning.
//
// A batch is a set of built handles whose products (each with its own
// right-hand sides) are captured once into a HIP graph and replayed with
// one launch.  With several right-hand sides the graph holds, per block of
// 16, one gather, phase-A, reduction, phase-B and scatter launch for all
// instances together (table-driven kernels over a work list of (instance,
// item) pairs, phase-A items of every instance ordered largest first), so
// small instances do not leave the machine idle; a handle listed twice
// goes to a second such round, since its work space is shared.  With one
// right-hand side the instances' own products are dealt to parallel graph
// branches.  The tuner picks, per handle, the work-item sizes by timing
// the candidates on the device.
#include "h2d_impl.h"

#include <algorithm>
#include <map>
#include <memory>
#include <vector>

namespace h2d {

constexpr int kBranches = 4;   // independent graph branches the instances are dealt to

struct Batch {
    std::vector<Handle*> hs;
    hipStream_t cap = nullptr;             // capture origin (default priority, like the branches)
    hipStream_t br[kBranches] = {};
    hipEvent_t fork = nullptr, join[kBranches] = {};
    std::vector<std::unique_ptr<MRBatchPlan>> plans;   // multi-RHS: one per round
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~Batch()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (int b = 0; b < kBranches; ++b) {
            if (join[b]) (void)hipEventDestroy(join[b]);
            if (br[b]) (void)hipStreamDestroy(br[b]);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

Batch* batch_create(Handle** hs, int count, int nrhs, double* const* x, double* const* y, const int64_t* ld)
{
    auto* B = new Batch();
    try {
        B->hs.assign(hs, hs + count);
        HIPCK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
        HIPCK(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
        for (int b = 0; b < kBranches; ++b) {
            HIPCK(hipStreamCreateWithFlags(&B->br[b], hipStreamNonBlocking));
            HIPCK(hipEventCreateWithFlags(&B->join[b], hipEventDisableTiming));
        }
        // one product per handle outside the capture allocates its work space
        for (int i = 0; i < count; ++i) {
            hs[i]->prof_on = false;
            launch_matvec(*hs[i], x[i], y[i], nrhs, ld[i], H2D_P_FP64, B->cap);
        }
        HIPCK(hipStreamSynchronize(B->cap));
        if (nrhs > 1) {
            // rounds: a handle listed k times appears in k rounds; handles
            // are dealt, largest first, to kBranches groups of similar total
            // size, each group of a round one table-driven plan on its
            // group's graph branch
            std::map<const Handle*, int> seen;
            std::vector<std::vector<int>> rounds;
            for (int i = 0; i < count; ++i) {
                const int r = seen[hs[i]]++;
                if ((int)rounds.size() <= r) rounds.emplace_back();
                rounds[r].push_back(i);
            }
            // every occurrence of a handle goes to the branch of its first
            // one (its work space is shared; a branch runs in order)
            std::map<const Handle*, int> branch_of;
            {
                std::vector<int> order(count);
                for (int i = 0; i < count; ++i) order[i] = i;
                std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a]->n > hs[b]->n; });
                int64_t load[kBranches] = {};
                for (int i : order) {
                    if (branch_of.count(hs[i])) continue;
                    const int g = (int)(std::min_element(load, load + kBranches) - load);
                    branch_of[hs[i]] = g;
                    load[g] += hs[i]->n;
                }
            }
            std::vector<int> plan_branch;
            for (const auto& members : rounds) {
                std::vector<std::vector<int>> groups(kBranches);
                for (int i : members) groups[branch_of[hs[i]]].push_back(i);
                for (int g = 0; g < kBranches; ++g) {
                    if (groups[g].empty()) continue;
                    std::vector<Handle*> h;
                    std::vector<MRIo> io;
                    for (int i : groups[g]) {
                        h.push_back(hs[i]);
                        io.push_back(MRIo{(uint64_t)(uintptr_t)x[i], (uint64_t)(uintptr_t)y[i], ld[i]});
                    }
                    B->plans.push_back(std::make_unique<MRBatchPlan>());
                    mr_plan(*B->plans.back(), h.data(), io.data(), (int)h.size(), B->cap);
                    plan_branch.push_back(g);
                }
            }
            // a later round of a group follows the earlier one on the same
            // branch (stream order)
            HIPCK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
            HIPCK(hipEventRecord(B->fork, B->cap));
            for (int b = 0; b < kBranches; ++b) HIPCK(hipStreamWaitEvent(B->br[b], B->fork, 0));
            for (size_t p = 0; p < B->plans.size(); ++p)
                for (int r0 = 0; r0 < nrhs; r0 += 16)
                    mr_plan_launch(*B->plans[p], r0, std::min(16, nrhs - r0), B->br[plan_branch[p]]);
            for (int b = 0; b < kBranches; ++b) {
                HIPCK(hipEventRecord(B->join[b], B->br[b]));
                HIPCK(hipStreamWaitEvent(B->cap, B->join[b], 0));
            }
            HIPCK(hipStreamEndCapture(B->cap, &B->graph));
            HIPCK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
            return B;
        }
        // A handle's work space is shared by its products, so every product
        // of one handle goes to the same branch; instances are dealt to the
        // branches by size so that the branches carry similar work.
        std::vector<int> order(count);
        for (int i = 0; i < count; ++i) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a]->n > hs[b]->n; });
        std::vector<int> branch(count, -1);
        int64_t load[kBranches] = {};
        for (int i : order) {
            for (int j = 0; j < count; ++j)
                if (branch[j] >= 0 && hs[j] == hs[i]) branch[i] = branch[j];
            if (branch[i] < 0) branch[i] = (int)(std::min_element(load, load + kBranches) - load);
            load[branch[i]] += hs[i]->n;
        }
        HIPCK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
        HIPCK(hipEventRecord(B->fork, B->cap));
        for (int b = 0; b < kBranches; ++b) HIPCK(hipStreamWaitEvent(B->br[b], B->fork, 0));
        for (int i : order) launch_matvec(*hs[i], x[i], y[i], nrhs, ld[i], H2D_P_FP64, B->br[branch[i]]);
        for (int b = 0; b < kBranches; ++b) {
            HIPCK(hipEventRecord(B->join[b], B->br[b]));
            HIPCK(hipStreamWaitEvent(B->cap, B->join[b], 0));
        }
        HIPCK(hipStreamEndCapture(B->cap, &B->graph));
        HIPCK(hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B->cap, &g);
        if (g) (void)hipGraphDestroy(g);
        delete B;
        throw;
    }
    return B;
}

void batch_launch(Batch* B, hipStream_t s) { HIPCK(hipGraphLaunch(B->exec, s)); }

void batch_destroy(Batch* B) { delete B; }

// which: 0 single-RHS phase-A item rows, 1 multi-RHS phase-A source-chunk
// rows, 2 single-RHS phase-B1 slice rows, 3 single-RHS phase-B2 leaf-chunk
// rows.
static void set_rows(Handle& H, int which, int32_t rows, hipStream_t s)
{
    if (which == 1) {
        H.mr_rows = rows;
        H.mr_cap = 0;   // rebuilt with the next multi-RHS product
    } else {
        (which == 0 ? H.a_rows : which == 2 ? H.b1_rows : H.b2_rows) = rows;
        if (which == 2) H.b1_rows_set = true;
        finalize(H, s);
    }
}

void set_item_rows(Handle& H, int which, int32_t rows, hipStream_t s) { set_rows(H, which, rows, s); }

// Time 5 products per candidate and keep the fastest; one right-hand side
// tunes phase A (128, 256, 512), then phase B1 (16, 32, 64), then phase B2
// (16, 32, 64); several tune the multi-RHS source chunks (128, 256, 512).
void autotune(Handle& H, int nrhs, hipStream_t s, int32_t* chosen, float* ms_out)
{
    const bool multi = nrhs > 1;
    const int64_t n = H.n;
    DBuf<double> x, y;
    x.alloc((size_t)n * nrhs);
    y.alloc((size_t)n * nrhs);
    HIPCK(hipMemsetAsync(x.p, 0, sizeof(double) * n * nrhs, s));
    hipEvent_t e0, e1;
    HIPCK(hipEventCreate(&e0));
    HIPCK(hipEventCreate(&e1));
    const bool prof = H.prof_on;
    H.prof_on = false;
    struct Knob {
        int which;
        int32_t cand[3];
    };
    const Knob single[3] = {{0, {128, 256, 512}}, {2, {16, 32, 64}}, {3, {16, 32, 64}}};
    const Knob mr[1] = {{1, {128, 256, 512}}};
    const Knob* knobs = multi ? mr : single;
    const int nk = multi ? 1 : 3;
    for (int kb = 0; kb < nk; ++kb) {
        float best = 1e30f;
        int32_t arg = knobs[kb].cand[0];
        for (int c = 0; c < 3; ++c) {
            set_rows(H, knobs[kb].which, knobs[kb].cand[c], s);
            launch_matvec(H, x.p, y.p, nrhs, n, H2D_P_FP64, s);   // warm-up, allocates
            HIPCK(hipEventRecord(e0, s));
            for (int r = 0; r < 5; ++r) launch_matvec(H, x.p, y.p, nrhs, n, H2D_P_FP64, s);
            HIPCK(hipEventRecord(e1, s));
            HIPCK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCK(hipEventElapsedTime(&ms, e0, e1));
            ms /= 5.f;
            if (ms_out) ms_out[3 * kb + c] = ms;
            if (ms < best) { best = ms; arg = knobs[kb].cand[c]; }
        }
        set_rows(H, knobs[kb].which, arg, s);
        if (chosen) chosen[kb] = arg;
    }
    if (multi && chosen) chosen[1] = chosen[2] = 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    H.prof_on = prof;
}

}  // namespace h2d
