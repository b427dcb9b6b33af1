// Batches across plans: the passes of many planned transforms run as a few
// persistent launches (the vector-loop rule of Section 4.2, applied across
// problems instead of within one).
//
// Pass k of every plan forms phase k; within a phase, passes that share a
// kernel family (precision, feature kind, workgroup size) become one launch of
// the persistent tile kernel over a device descriptor list.  Tiles are numbered
// item by item, items ordered by line length, largest first, and workgroups
// pop tile indices from a counter, so long lines start early and short ones
// fill the tail.  Phases run in order on the stream, so pass k+1 of a plan
// always sees pass k complete.  Counters are cleared by a kernel (not a memset)
// so that the whole sequence can be captured in a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "plan.h"

namespace mfft {

extern int g_num_cus;

struct BatchGroup {
    int prec = 0, kind = 0, block = 0;
    size_t lds = 0;
    int grid = 0;
    int nitems = 0;
    int64_t tiles = 0;
    PassArgs *d_items = nullptr;
    int64_t *d_prefix = nullptr;
    unsigned long long *d_counter = nullptr;
};

struct BatchStep {          // one launch: a group, or a copy pass
    bool copy = false;
    CopyArgs c{};
    int group = -1;
};

}  // namespace mfft

struct mfft_batch_s {
    std::vector<mfft::BatchGroup> groups;
    std::vector<mfft::BatchStep> steps;
    void *dev_mem = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t tiles = 0;
};

namespace mfft {

static int enqueue_steps(mfft_batch_s *b, hipStream_t s)
{
    for (const BatchStep &st : b->steps) {
        hipError_t e;
        if (st.copy) {
            e = launch_copy(st.c, s);
        } else {
            const BatchGroup &g = b->groups[st.group];
            e = launch_zero_u64(g.d_counter, 1, s);
            if (e == hipSuccess)
                e = launch_batch(g.d_items, g.d_prefix, g.nitems, g.d_counter, g.prec, g.kind,
                                 g.block, g.grid, g.lds, s);
        }
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    return MFFT_OK;
}

static void batch_free(mfft_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->dev_mem) (void)hipFree(b->dev_mem);
    delete b;
}

}  // namespace mfft

using namespace mfft;

extern "C" {

int mfft_batch_create(mfft_batch *out, int count, const mfft_plan *plans, const void *const *ins,
                      void *const *outs, unsigned flags, void *hip_stream)
{
    if (!out || count < 0 || (count > 0 && (!plans || !ins || !outs)))
        return fail(MFFT_EINVAL, "bad batch arguments");
    *out = nullptr;
    std::set<const void *> scratch_seen;
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return fail(MFFT_EINVAL, "NULL plan in batch");
        const PlanImpl *p = &plans[i]->impl;
        if (!p->prob.empty && (!ins[i] || !outs[i])) return fail(MFFT_EINVAL, "NULL buffer in batch");
        if (p->prob.inplace != (ins[i] == outs[i]))
            return fail(MFFT_EALIGN, "batch item buffers contradict the plan's in-place rule");
        if (p->scratch) {
            if (!scratch_seen.insert(p->scratch).second)
                return fail(MFFT_EINVAL, "a plan with scratch appears twice in one batch");
        }
    }
    mfft_batch_s *b = new (std::nothrow) mfft_batch_s();
    if (!b) return fail(MFFT_ENOMEM, "host allocation failed");

    // collect (phase, family) -> items
    struct Item {
        PassArgs a;
        int64_t n;
    };
    using Key = std::tuple<int, int, int, int>;   // phase, prec, kind, block
    std::map<Key, std::vector<Item>> fam;
    std::map<Key, size_t> fam_lds;
    std::map<int, std::vector<CopyArgs>> copies;
    int nphase = 0;
    for (int i = 0; i < count; ++i) {
        const PlanImpl *p = &plans[i]->impl;
        for (size_t k = 0; k < p->passes.size(); ++k) {
            const Pass &ps = p->passes[k];
            nphase = std::max(nphase, (int)k + 1);
            if (ps.kind == 1) {
                copies[(int)k].push_back(resolve_copy(p, ps, ins[i], outs[i], p->scratch));
                continue;
            }
            PassArgs a = resolve_pass(p, ps, ins[i], outs[i], p->scratch);
            if (a.ntiles <= 0) continue;
            const int block = a.bt * a.tpt;
            const Key key{(int)k, p->prob.prec, pass_kind(a.flags), block};
            fam[key].push_back({a, (int64_t)a.n});
            fam_lds[key] = std::max(fam_lds[key], generic_lds_bytes(ps));
        }
    }
    // device layout: per group items[], prefix[], counter
    size_t bytes = 0;
    std::vector<std::pair<Key, std::vector<Item>>> order(fam.begin(), fam.end());
    for (auto &kv : order) {
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [](const Item &x, const Item &y) { return x.n > y.n; });
        bytes += kv.second.size() * sizeof(PassArgs) + 256;
        bytes += (kv.second.size() + 1) * sizeof(int64_t) + 256;
        bytes += 256;
    }
    std::vector<unsigned char> host(bytes ? bytes : 1);
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = (off + 255) / 256 * 256;
        off = o + n;
        return o;
    };
    struct Place {
        size_t items, prefix, counter;
    };
    std::vector<Place> places;
    for (auto &kv : order) {
        Place pl;
        pl.items = take(kv.second.size() * sizeof(PassArgs));
        pl.prefix = take((kv.second.size() + 1) * sizeof(int64_t));
        pl.counter = take(sizeof(unsigned long long));
        places.push_back(pl);
        PassArgs *items = (PassArgs *)(host.data() + pl.items);
        int64_t *prefix = (int64_t *)(host.data() + pl.prefix);
        prefix[0] = 0;
        for (size_t j = 0; j < kv.second.size(); ++j) {
            items[j] = kv.second[j].a;
            prefix[j + 1] = prefix[j] + kv.second[j].a.ntiles;
        }
    }
    if (off && hipMalloc(&b->dev_mem, off) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return fail(MFFT_ENOMEM, "batch descriptor allocation failed");
    }
    hipStream_t s = (hipStream_t)hip_stream;
    if (off && hipMemcpy(b->dev_mem, host.data(), off, hipMemcpyHostToDevice) != hipSuccess) {
        batch_free(b);
        return fail(MFFT_EHIP, "batch descriptor upload failed");
    }
    for (size_t gi = 0; gi < order.size(); ++gi) {
        const Key &key = order[gi].first;
        BatchGroup g;
        g.prec = std::get<1>(key);
        g.kind = std::get<2>(key);
        g.block = std::get<3>(key);
        g.lds = fam_lds[key];
        g.nitems = (int)order[gi].second.size();
        const int64_t *prefix = (const int64_t *)(host.data() + places[gi].prefix);
        g.tiles = prefix[g.nitems];
        b->tiles += g.tiles;
        const int64_t resident =
            (int64_t)batch_blocks_per_cu(g.prec, g.kind, g.block, g.lds) * g_num_cus;
        g.grid = (int)std::max<int64_t>(1, std::min<int64_t>(g.tiles, resident));
        char *base = (char *)b->dev_mem;
        g.d_items = (PassArgs *)(base + places[gi].items);
        g.d_prefix = (int64_t *)(base + places[gi].prefix);
        g.d_counter = (unsigned long long *)(base + places[gi].counter);
        b->groups.push_back(g);
    }
    for (int k = 0; k < nphase; ++k) {
        for (const CopyArgs &c : copies[k]) {
            BatchStep st;
            st.copy = true;
            st.c = c;
            b->steps.push_back(st);
        }
        for (size_t gi = 0; gi < order.size(); ++gi)
            if (std::get<0>(order[gi].first) == k) {
                BatchStep st;
                st.group = (int)gi;
                b->steps.push_back(st);
            }
    }
    if (flags & MFFT_BATCH_GRAPH) {
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
        int rc = e == hipSuccess ? enqueue_steps(b, b->cap_stream) : MFFT_EHIP;
        hipError_t e2 = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess && rc == MFFT_OK) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess || rc != MFFT_OK) {
            batch_free(b);
            return fail(MFFT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
    }
    (void)s;
    *out = b;
    return MFFT_OK;
}

int mfft_batch_execute(mfft_batch batch, void *hip_stream)
{
    if (!batch) return fail(MFFT_EINVAL, "batch is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    if (batch->exec) {
        hipError_t e = hipGraphLaunch(batch->exec, s);
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("graph launch: ") + hipGetErrorString(e));
        return MFFT_OK;
    }
    return enqueue_steps(batch, s);
}

int mfft_batch_info(mfft_batch batch, int *launches, int64_t *tiles)
{
    if (!batch) return fail(MFFT_EINVAL, "batch is NULL");
    if (launches) {
        int n = 0;
        for (const BatchStep &st : batch->steps) n += st.copy ? 1 : 2;   // counter clear + kernel
        *launches = n;
    }
    if (tiles) *tiles = batch->tiles;
    return MFFT_OK;
}

int mfft_batch_destroy(mfft_batch batch)
{
    if (!batch) return MFFT_OK;
    batch_free(batch);
    return MFFT_OK;
}

}  // extern "C"
