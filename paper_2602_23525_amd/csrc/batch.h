// Batch layout shared by mfft_batch_* and the request server: the host image
// of the descriptor lists, prefix sums and tile-to-item tables, and the launch
// sequence.
#pragma once
#include <vector>

#include "plan.h"

namespace mfft {

struct BatchItem {
    const PlanImpl *plan;
    const void *in;
    void *out;
    void *scratch;   // the plan's scratch or a caller-provided region of the same size
};

struct BatchGroup {
    int leaf_n = 0, leaf_mode = 0;   // leaf_n > 0: a batched leaf launch (one tile per workgroup)
    int prec = 0, kind = 0, block = 0;
    size_t lds = 0;
    int grid = 0;
    int nitems = 0;
    int64_t tiles = 0;
    size_t items_off = 0, prefix_off = 0;   // offsets in the image
    size_t owner_off = 0;   // the item of each tile (int32)
};

struct BatchStep {   // one launch: a group, a copy pass, a real-data step or a transpose
    bool copy = false;
    CopyArgs c{};
    bool real = false;
    RealArgs r{};
    bool transpose = false;
    TransposeArgs t{};
    bool permute = false;
    PermuteArgs pm{};
    bool leaf = false;   // a specialized leaf pass with a real-data fusion
    PassArgs a{};
    int leaf_variant = 0, leaf_grid = 0;
    int prec = 0;
    int group = -1;
    int phase = 0;       // pass index of the plans: phases run in order
    int lane = 0;        // concurrent lane of the phase (0: the caller's stream)
    double cost = 0;     // complex elements the launch moves (lane balancing)
};

struct BatchLayout {
    std::vector<unsigned char> host;   // device image (upload `bytes` of it)
    size_t bytes = 0;
    std::vector<BatchGroup> groups;
    std::vector<BatchStep> steps;
    int64_t tiles = 0;
};

// Lanes per phase that build_batch_layout balances the steps over.
constexpr int kBatchLanes = 4;

int build_batch_layout(const std::vector<BatchItem> &items, BatchLayout *L);
// Launch the sequence with the image resident at `dev`.  With `aux`
// (kBatchLanes - 1 streams) and `ev` (kBatchLanes events), the steps of a
// phase, which touch different plans' buffers, run as concurrent lanes: the
// auxiliary streams wait for the phase's start on s, and s waits for their
// ends before the next phase (under graph capture: parallel branches).
int enqueue_batch_layout(const BatchLayout &L, char *dev, hipStream_t s,
                         const hipStream_t *aux = nullptr, hipEvent_t *ev = nullptr);
int batch_launch_count(const BatchLayout &L);

}  // namespace mfft
