// Batches across plans: the passes of many planned transforms run as a few
// launches (the vector-loop rule of Section 4.2, applied across problems
// instead of within one).
//
// Pass k of every plan forms phase k; within a phase, passes that share a
// kernel family (precision, feature kind, workgroup-size class) become one
// launch of the tile kernel over a device descriptor list, one workgroup per
// tile.  Tiles are numbered item by item, items ordered by line length,
// largest first, and each workgroup finds its tile's item in a tile-to-item
// table, so long lines start early and short ones fill the tail.  Phases run
// in order on the stream, so pass k+1 of a plan always sees pass k complete.
// The sequence holds kernel launches only, so it can be captured in a HIP
// graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <set>
#include <tuple>
#include <vector>

#include "batch.h"

namespace mfft {

extern size_t g_lds_budget;

// Retile a pass for a workgroup-size class: 256, 512 or 1024 threads, with
// more lines per tile so few lanes idle in the class (tiles kept <= 64 KB).
static int widen(const Pass &ps, PassArgs *a, size_t *lds)
{
    const int maxb = ps.prec || ps.emax > 16 ? 512 : 1024;
    int block = std::min(256, maxb);
    while (block < a->bt * a->tpt) block *= 2;
    Pass wide = ps;
    int bt = a->bt;
    if (a->load_mode == kModeRow && a->store_mode == kModeRow) {
        // row tiles take any line count: as many as the class holds
        while ((bt + 1) * a->tpt <= block && bt + 1 <= a->vn) {
            wide.a.bt = bt + 1;
            if (generic_lds_bytes(wide) > std::min<size_t>(g_lds_budget, 65536)) break;
            ++bt;
        }
    } else {
        while (bt * 2 * a->tpt <= block && bt * 2 <= a->vn) {
            wide.a.bt = bt * 2;
            if (generic_lds_bytes(wide) > std::min<size_t>(g_lds_budget, 65536)) break;
            bt *= 2;
        }
    }
    wide.a.bt = bt;
    if (bt != a->bt) {
        const int64_t outer = a->ntiles / a->ntiles_inner;
        a->bt = bt;
        int l = 0;
        while ((1 << l) < bt) ++l;
        a->bt_log2 = l;
        a->ntiles_inner = (a->vn + bt - 1) / bt;
        a->ntiles = a->ntiles_inner * outer;
    }
    *lds = generic_lds_bytes(wide);
    return block;
}

int build_batch_layout(const std::vector<BatchItem> &items, BatchLayout *L)
{
    struct Item {
        PassArgs a;
        int64_t n;
    };
    using Key = std::tuple<int, int, int, int>;   // phase, prec, kind, block
    std::map<Key, std::vector<Item>> fam;
    std::map<Key, size_t> fam_lds;
    std::map<int, std::vector<CopyArgs>> copies;
    std::map<int, std::vector<std::pair<RealArgs, int>>> reals;
    std::map<int, std::vector<TransposeArgs>> transposes;
    std::map<int, std::vector<PermuteArgs>> permutes;
    std::map<int, std::vector<BatchStep>> leaves;
    // specialized leaf passes: one launch per phase, precision, length and tile kind
    using LKey = std::tuple<int, int, int, int>;   // phase, prec, n, mode
    std::map<LKey, std::vector<PassArgs>> leaffam;
    int nphase = 0;
    for (const BatchItem &it : items) {
        const PlanImpl *p = it.plan;
        for (size_t k = 0; k < p->passes.size(); ++k) {
            const Pass &ps = p->passes[k];
            nphase = std::max(nphase, (int)k + 1);
            if (ps.kind == 1) {
                copies[(int)k].push_back(resolve_copy(p, ps, it.in, it.out, it.scratch));
                continue;
            }
            if (ps.kind == 2) {
                reals[(int)k].push_back({resolve_real(p, ps, it.in, it.out, it.scratch), ps.prec});
                continue;
            }
            if (ps.kind == 3) {
                transposes[(int)k].push_back(resolve_transpose(p, ps, it.in, it.out, it.scratch));
                continue;
            }
            if (ps.kind == 4) {
                permutes[(int)k].push_back(resolve_permute(p, ps, it.in, it.out, it.scratch));
                continue;
            }
            PassArgs a = resolve_pass(p, ps, it.in, it.out, it.scratch);
            if (a.ntiles <= 0) continue;
            if (a.flags & (PF_R2C | PF_C2R)) {
                // the fused split/combine exists only in the specialized leaf kernel
                BatchStep st;
                st.leaf = true;
                st.a = a;
                st.leaf_variant = ps.variant;
                st.leaf_grid = (int)ps.grid;
                st.prec = ps.prec;
                leaves[(int)k].push_back(st);
                continue;
            }
            if (ps.kernel == 1 && a.vn >= a.bt) {
                // full leaf tiles: the batched leaf launch (a pass with fewer
                // lines than a leaf tile goes to the tile kernel, whose tiles
                // shrink to the lines present)
                leaffam[LKey{(int)k, ps.prec, (int)a.n, leaf_batch_mode(a.flags)}].push_back(a);
                continue;
            }
            size_t lds = 0;
            const int block = widen(ps, &a, &lds);
            const Key key{(int)k, p->prob.prec,
                          pass_kind(a.flags) + (ps.emax > 16 ? kWideKind : 0), block};
            fam[key].push_back({a, (int64_t)a.n});
            fam_lds[key] = std::max(fam_lds[key], lds);
        }
    }
    std::vector<std::pair<Key, std::vector<Item>>> order(fam.begin(), fam.end());
    size_t bytes = 512;
    for (auto &kv : order) {
        std::stable_sort(kv.second.begin(), kv.second.end(),
                         [](const Item &x, const Item &y) { return x.n > y.n; });
        bytes += kv.second.size() * sizeof(PassArgs) + 256;
        bytes += (kv.second.size() + 1) * sizeof(int64_t) + 256;
        int64_t t = 0;
        for (const Item &it : kv.second) t += it.a.ntiles;
        if (t > 0x7fffffffLL) return fail(MFFT_ENOTSUP, "batched launch too large");
        bytes += (size_t)t * sizeof(int32_t) + 256;
    }
    for (auto &kv : leaffam) {
        bytes += kv.second.size() * sizeof(PassArgs) + 256;
        bytes += (kv.second.size() + 1) * sizeof(int64_t) + 256;
        int64_t t = 0;
        for (const PassArgs &a : kv.second) t += a.ntiles;
        if (t > 0x7fffffffLL) return fail(MFFT_ENOTSUP, "batched leaf launch too large");
        bytes += (size_t)t * sizeof(int32_t) + 256;
    }
    L->host.assign(bytes, 0);
    size_t off = 0;
    auto take = [&](size_t n) {
        size_t o = (off + 255) / 256 * 256;
        off = o + n;
        return o;
    };
    L->groups.clear();
    L->steps.clear();
    L->tiles = 0;
    for (size_t gi = 0; gi < order.size(); ++gi) {
        auto &kv = order[gi];
        BatchGroup g;
        g.items_off = take(kv.second.size() * sizeof(PassArgs));
        g.prefix_off = take((kv.second.size() + 1) * sizeof(int64_t));
        PassArgs *dst = (PassArgs *)(L->host.data() + g.items_off);
        int64_t *prefix = (int64_t *)(L->host.data() + g.prefix_off);
        prefix[0] = 0;
        for (size_t j = 0; j < kv.second.size(); ++j) {
            dst[j] = kv.second[j].a;
            prefix[j + 1] = prefix[j] + kv.second[j].a.ntiles;
        }
        g.prec = std::get<1>(kv.first);
        g.kind = std::get<2>(kv.first);
        g.block = std::get<3>(kv.first);
        g.lds = fam_lds[kv.first];
        g.nitems = (int)kv.second.size();
        g.tiles = prefix[g.nitems];
        g.owner_off = take((size_t)g.tiles * sizeof(int32_t));
        int32_t *owner = (int32_t *)(L->host.data() + g.owner_off);
        for (int j = 0; j < g.nitems; ++j)
            for (int64_t t = prefix[j]; t < prefix[j + 1]; ++t) owner[t] = j;
        L->tiles += g.tiles;
        g.grid = (int)g.tiles;
        L->groups.push_back(g);
    }
    std::map<int, std::vector<int>> leaf_groups;   // phase -> group indices
    for (auto &kv : leaffam) {
        BatchGroup g;
        g.items_off = take(kv.second.size() * sizeof(PassArgs));
        g.prefix_off = take((kv.second.size() + 1) * sizeof(int64_t));
        PassArgs *dst = (PassArgs *)(L->host.data() + g.items_off);
        int64_t *prefix = (int64_t *)(L->host.data() + g.prefix_off);
        prefix[0] = 0;
        for (size_t j = 0; j < kv.second.size(); ++j) {
            dst[j] = kv.second[j];
            prefix[j + 1] = prefix[j] + kv.second[j].ntiles;
        }
        g.prec = std::get<1>(kv.first);
        g.leaf_n = std::get<2>(kv.first);
        g.leaf_mode = std::get<3>(kv.first);
        g.nitems = (int)kv.second.size();
        g.tiles = prefix[g.nitems];
        g.grid = (int)g.tiles;
        g.owner_off = take((size_t)g.tiles * sizeof(int32_t));
        int32_t *owner = (int32_t *)(L->host.data() + g.owner_off);
        for (int j = 0; j < g.nitems; ++j)
            for (int64_t t = prefix[j]; t < prefix[j + 1]; ++t) owner[t] = j;
        L->tiles += g.tiles;
        leaf_groups[std::get<0>(kv.first)].push_back((int)L->groups.size());
        L->groups.push_back(g);
    }
    L->bytes = off;
    for (int k = 0; k < nphase; ++k) {
        for (const CopyArgs &c : copies[k]) {
            BatchStep st;
            st.copy = true;
            st.c = c;
            L->steps.push_back(st);
        }
        for (const BatchStep &st : leaves[k]) L->steps.push_back(st);
        for (const auto &rp : reals[k]) {
            BatchStep st;
            st.real = true;
            st.r = rp.first;
            st.prec = rp.second;
            L->steps.push_back(st);
        }
        for (const TransposeArgs &t : transposes[k]) {
            BatchStep st;
            st.transpose = true;
            st.t = t;
            L->steps.push_back(st);
        }
        for (const PermuteArgs &pa : permutes[k]) {
            BatchStep st;
            st.permute = true;
            st.pm = pa;
            L->steps.push_back(st);
        }
        for (int gi : leaf_groups[k]) {
            BatchStep st;
            st.group = gi;
            L->steps.push_back(st);
        }
        for (size_t gi = 0; gi < order.size(); ++gi)
            if (std::get<0>(order[gi].first) == k) {
                BatchStep st;
                st.group = (int)gi;
                L->steps.push_back(st);
            }
    }
    // phases, costs and lanes: within a phase the steps are balanced over
    // kBatchLanes lanes by the elements they move, largest first
    {
        size_t i = 0;
        for (int k = 0; k < nphase; ++k) {
            const size_t n_k = copies[k].size() + leaves[k].size() + reals[k].size() +
                               transposes[k].size() + permutes[k].size() + leaf_groups[k].size();
            size_t n_g = 0;
            for (size_t gi = 0; gi < order.size(); ++gi) n_g += std::get<0>(order[gi].first) == k;
            const size_t end = i + n_k + n_g;
            std::vector<size_t> idx;
            for (size_t j = i; j < end; ++j) {
                BatchStep &st = L->steps[j];
                st.phase = k;
                double c = 1.0;
                auto pass_cost = [](const PassArgs &a) {
                    return (double)a.ntiles * (double)a.bt * (double)a.n;
                };
                if (st.group >= 0) {
                    const BatchGroup &g = L->groups[st.group];
                    const PassArgs *it = (const PassArgs *)(L->host.data() + g.items_off);
                    c = 0;
                    for (int m = 0; m < g.nitems; ++m) c += pass_cost(it[m]);
                } else if (st.leaf) {
                    c = pass_cost(st.a);
                } else if (st.copy) {
                    c = (double)st.c.total;
                }
                st.cost = c;
                idx.push_back(j);
            }
            std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
                return L->steps[x].cost > L->steps[y].cost;
            });
            double load[kBatchLanes] = {};
            for (size_t j : idx) {
                int best = 0;
                for (int l = 1; l < kBatchLanes; ++l)
                    if (load[l] < load[best]) best = l;
                L->steps[j].lane = best;
                load[best] += L->steps[j].cost;
            }
            i = end;
        }
    }
    return MFFT_OK;
}

int enqueue_batch_layout(const BatchLayout &L, char *dev, hipStream_t s, const hipStream_t *aux,
                         hipEvent_t *ev)
{
    const bool lanes = aux && ev;
    int phase = -1;
    bool used[kBatchLanes] = {};
    auto join = [&]() -> hipError_t {
        // s waits for the lanes that ran in the phase
        for (int l = 1; l < kBatchLanes; ++l) {
            if (!used[l]) continue;
            hipError_t e = hipEventRecord(ev[l], aux[l - 1]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, ev[l], 0);
            if (e != hipSuccess) return e;
            used[l] = false;
        }
        return hipSuccess;
    };
    for (const BatchStep &st : L.steps) {
        hipError_t e;
        hipStream_t q = s;
        if (lanes) {
            if (st.phase != phase) {
                e = join();
                if (e == hipSuccess) e = hipEventRecord(ev[0], s);   // the phase starts
                if (e != hipSuccess)
                    return fail(MFFT_EHIP, std::string("batch lanes: ") + hipGetErrorString(e));
                phase = st.phase;
            }
            if (st.lane > 0) {
                q = aux[st.lane - 1];
                if (!used[st.lane]) {
                    e = hipStreamWaitEvent(q, ev[0], 0);
                    if (e != hipSuccess)
                        return fail(MFFT_EHIP, std::string("batch lanes: ") + hipGetErrorString(e));
                    used[st.lane] = true;
                }
            }
        }
        if (st.copy) {
            e = launch_copy(st.c, q);
        } else if (st.real) {
            e = launch_real(st.r, st.prec, q);
        } else if (st.transpose) {
            e = launch_transpose_sq(st.t, q);
        } else if (st.permute) {
            e = launch_permute_items(st.pm, q);
        } else if (st.leaf) {
            e = launch_leaf(st.a, st.prec, st.a.n, st.leaf_variant, st.leaf_grid, q);
        } else if (L.groups[st.group].leaf_n > 0) {
            const BatchGroup &g = L.groups[st.group];
            e = launch_leaf_batch((const PassArgs *)(dev + g.items_off),
                                  (const int64_t *)(dev + g.prefix_off),
                                  (const int32_t *)(dev + g.owner_off), g.tiles, g.prec, g.leaf_n,
                                  g.leaf_mode, q);
        } else {
            const BatchGroup &g = L.groups[st.group];
            e = launch_batch((const PassArgs *)(dev + g.items_off),
                             (const int64_t *)(dev + g.prefix_off),
                             (const int32_t *)(dev + g.owner_off), g.tiles, g.prec, g.kind,
                             g.block, g.lds, q);
            if (e != hipSuccess)
                return fail(MFFT_EHIP, std::string("batch launch (block ") + std::to_string(g.block) +
                                           ", lds " + std::to_string(g.lds) + ", grid " +
                                           std::to_string(g.grid) + "): " + hipGetErrorString(e));
        }
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
    }
    if (lanes) {
        hipError_t e = join();
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("batch lanes: ") + hipGetErrorString(e));
    }
    return MFFT_OK;
}

int batch_launch_count(const BatchLayout &L)
{
    return (int)L.steps.size();
}

}  // namespace mfft

struct mfft_batch_s {
    mfft::BatchLayout layout;
    void *dev_mem = nullptr;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    // the concurrent lanes of a phase (default priority, non-blocking)
    hipStream_t aux[mfft::kBatchLanes - 1] = {};
    hipEvent_t ev[mfft::kBatchLanes] = {};
    bool lanes = false;
};

namespace mfft {

static void batch_free(mfft_batch_s *b)
{
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (hipStream_t q : b->aux)
        if (q) (void)hipStreamDestroy(q);
    for (hipEvent_t e : b->ev)
        if (e) (void)hipEventDestroy(e);
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
    std::vector<BatchItem> items;
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
        items.push_back({p, ins[i], outs[i], p->scratch});
    }
    mfft_batch_s *b = new (std::nothrow) mfft_batch_s();
    if (!b) return fail(MFFT_ENOMEM, "host allocation failed");
    int rc = build_batch_layout(items, &b->layout);
    if (rc) {
        batch_free(b);
        return rc;
    }
    if (b->layout.bytes && hipMalloc(&b->dev_mem, b->layout.bytes) != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return fail(MFFT_ENOMEM, "batch descriptor allocation failed");
    }
    if (b->layout.bytes &&
        hipMemcpy(b->dev_mem, b->layout.host.data(), b->layout.bytes, hipMemcpyHostToDevice) !=
            hipSuccess) {
        batch_free(b);
        return fail(MFFT_EHIP, "batch descriptor upload failed");
    }
    (void)hip_stream;
    {
        hipError_t e = hipSuccess;
        for (hipStream_t &q : b->aux)
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&q, hipStreamNonBlocking);
        for (hipEvent_t &ev : b->ev)
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            batch_free(b);
            return fail(MFFT_EHIP, std::string("batch lanes: ") + hipGetErrorString(e));
        }
        b->lanes = true;
    }
    if (flags & MFFT_BATCH_GRAPH) {
        hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
        rc = e == hipSuccess ? enqueue_batch_layout(b->layout, (char *)b->dev_mem, b->cap_stream,
                                                    b->aux, b->ev)
                             : MFFT_EHIP;
        if (e == hipSuccess) {
            hipError_t e2 = hipStreamEndCapture(b->cap_stream, &b->graph);
            if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess && rc == MFFT_OK)
            e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e != hipSuccess || rc != MFFT_OK) {
            batch_free(b);
            return fail(MFFT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
    }
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
    return enqueue_batch_layout(batch->layout, (char *)batch->dev_mem, s, batch->aux, batch->ev);
}

int mfft_batch_info(mfft_batch batch, int *launches, int64_t *tiles)
{
    if (!batch) return fail(MFFT_EINVAL, "batch is NULL");
    if (launches) *launches = batch_launch_count(batch->layout);
    if (tiles) *tiles = batch->layout.tiles;
    return MFFT_OK;
}

int mfft_batch_destroy(mfft_batch batch)
{
    if (!batch) return MFFT_OK;
    batch_free(batch);
    return MFFT_OK;
}

}  // extern "C"
