// Measure mode and wisdom (Section 4.3, "The FFTW planner"): build the plan
// for each applicable choice, time it, keep the fastest; choices can be saved
// and loaded later.  Each choice is optimized on its own, independently of
// the others -- the dynamic-programming approximation the paper describes.
// Two levels of choices:
//   structure, per transform length: the radix sequence and lines per tile of
//     a one-pass generic leaf, the split of a two-pass Cooley-Tukey length,
//     Rader or Bluestein for a prime and Bluestein's convolution length
//     (each candidate is a rebuilt plan, timed whole);
//   kernel variant, per pass of the specialized leaf kernel: prefetch,
//     occupancy floor, non-temporal access, grid kind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <map>
#include <sstream>
#include <vector>

#include "plan.h"

namespace mfft {

// Offsets (in elements) a pass can touch on its read (which = 0) or write side.
static void pass_extent(const Pass &ps, int which, int64_t *lo, int64_t *hi)
{
    const PassArgs &a = ps.a;
    int64_t l = 0, h = 0;
    auto add = [&](int64_t n, int64_t s) {
        if (n <= 1) return;
        const int64_t e = (n - 1) * s;
        if (e < 0) l += e;
        else h += e;
    };
    add(a.n, which ? a.os : a.is);
    add(a.vn, which ? a.vos : a.vis);
    for (int d = 0; d < a.nouter; ++d) add(a.on[d], which ? a.oos[d] : a.ois[d]);
    *lo = l;
    *hi = h;
}

static const int kCandVariants[] = {24, 25, 29, 8, 9, 0};

// Extent of the problem's input (which = 0) or output tensor in elements.
static void problem_extent(const Problem &pr, int which, int64_t *lo, int64_t *hi)
{
    int64_t l = 0, h = 0;
    for (const std::vector<Dim> *V : {&pr.N, &pr.V})
        for (const Dim &d : *V) {
            if (d.n <= 1) continue;
            const int64_t e = (d.n - 1) * (which ? d.os : d.is);
            if (e < 0) l += e;
            else h += e;
        }
    *lo = l;
    *hi = h;
}

// Average time of the plan as it stands on the given buffers (ms), or < 0.
static float time_plan(const PlanImpl *p, void *in, void *out, hipEvent_t e0, hipEvent_t e1)
{
    void *scratch = nullptr;
    if (p->scratch_bytes && hipMalloc(&scratch, p->scratch_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return -1.f;
    }
    float ms = -1.f;
    int rc = MFFT_OK;
    for (int w = 0; w < 2 && rc == MFFT_OK; ++w) rc = run_plan(p, in, out, scratch, p->stream);
    if (rc == MFFT_OK) {
        const int reps = 5;
        (void)hipEventRecord(e0, p->stream);
        for (int r = 0; r < reps && rc == MFFT_OK; ++r) rc = run_plan(p, in, out, scratch, p->stream);
        (void)hipEventRecord(e1, p->stream);
        if (rc == MFFT_OK && hipEventSynchronize(e1) == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess)
            ms /= reps;
        else
            ms = -1.f;
    }
    (void)hipStreamSynchronize(p->stream);
    if (scratch) (void)hipFree(scratch);
    return ms;
}

int measure_structure(PlanImpl *p)
{
    if (p->prob.kind != 0 || p->prob.empty) return MFFT_OK;
    std::vector<int64_t> lengths;
    for (const Dim &d : p->prob.N)
        if (std::find(lengths.begin(), lengths.end(), d.n) == lengths.end()) lengths.push_back(d.n);
    std::vector<std::pair<int64_t, std::vector<StructChoice>>> todo;
    for (int64_t n : lengths) {
        auto c = structure_candidates(p, n);
        if (c.size() > 1) todo.push_back({n, c});
        else if (!c[0].empty()) p->overrides[n] = c[0];   // nothing to time: the estimate's
    }
    if (todo.empty()) return rebuild_plan(p);
    const size_t eb = p->prob.prec ? 16 : 8;
    int64_t ilo, ihi, olo, ohi;
    problem_extent(p->prob, 0, &ilo, &ihi);
    problem_extent(p->prob, 1, &olo, &ohi);
    if (p->prob.inplace) {
        ilo = olo = std::min(ilo, olo);
        ihi = ohi = std::max(ihi, ohi);
    }
    const size_t ib = (size_t)(ihi - ilo + 1) * eb, ob = (size_t)(ohi - olo + 1) * eb;
    const size_t cap = (size_t)1 << 30;
    if (ib > cap || ob > cap) return MFFT_OK;   // too large to time here: estimate
    void *bin = nullptr, *bout = nullptr;
    if (hipMalloc(&bin, ib) != hipSuccess ||
        (!p->prob.inplace && hipMalloc(&bout, ob) != hipSuccess)) {
        (void)hipGetLastError();
        if (bin) (void)hipFree(bin);
        return MFFT_OK;
    }
    (void)hipMemsetAsync(bin, 0, ib, p->stream);
    char *in = (char *)bin - ilo * (int64_t)eb;
    char *out = p->prob.inplace ? in : (char *)bout - olo * (int64_t)eb;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipFree(bin);
        if (bout) (void)hipFree(bout);
        return fail(MFFT_EHIP, "event creation failed");
    }
    auto signature = [](const PlanImpl *q) {
        std::string sig;
        for (const Pass &ps : q->passes) sig += ps.desc + "\n";
        return sig;
    };
    int rc = MFFT_OK;
    for (auto &job : todo) {
        const int64_t n = job.first;
        StructChoice best = job.second[0];   // the estimate's choice
        p->overrides.erase(n);
        rc = rebuild_plan(p);
        if (rc) break;
        float best_ms = time_plan(p, in, out, e0, e1);
        std::vector<std::string> seen = {signature(p)};
        for (size_t i = 1; i < job.second.size(); ++i) {
            p->overrides[n] = job.second[i];
            if (rebuild_plan(p) != MFFT_OK) continue;   // candidate has no plan here
            const std::string sig = signature(p);
            if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;   // same plan
            seen.push_back(sig);
            const float ms = time_plan(p, in, out, e0, e1);
            // a candidate replaces the estimate only when clearly faster
            if (ms > 0 && (best_ms <= 0 || ms < 0.97f * best_ms)) {
                best_ms = ms;
                best = job.second[i];
            }
        }
        // kept spelled out (also when the estimate's won), for the wisdom text
        if (best.empty()) p->overrides.erase(n);
        else p->overrides[n] = best;
    }
    if (rc == MFFT_OK) rc = rebuild_plan(p);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(bin);
    if (bout) (void)hipFree(bout);
    return rc;
}

int measure_plan(PlanImpl *p)
{
    const size_t eb = p->prob.prec ? 16 : 8;
    const size_t cap = (size_t)2 << 30;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(MFFT_EHIP, "event creation failed");
    int rc = MFFT_OK;
    for (Pass &ps : p->passes) {
        // column tiles have one configuration
        if (ps.kind != 0 || ps.kernel != 1 || (ps.a.flags & PF_LEAF_COL)) continue;
        int64_t ilo, ihi, olo, ohi;
        pass_extent(ps, 0, &ilo, &ihi);
        pass_extent(ps, 1, &olo, &ohi);
        const size_t ib = (size_t)(ihi - ilo + 1) * eb, ob = (size_t)(ohi - olo + 1) * eb;
        if (ib > cap || ob > cap) continue;
        void *bin = nullptr, *bout = nullptr;
        if (hipMalloc(&bin, ib) != hipSuccess || hipMalloc(&bout, ob) != hipSuccess) {
            (void)hipGetLastError();
            if (bin) (void)hipFree(bin);
            continue;
        }
        (void)hipMemsetAsync(bin, 0, ib, p->stream);
        float best = 1e30f;
        LeafTune best_t = {ps.variant, ps.persistent};
        for (int v : kCandVariants) {
            for (int pers = 0; pers < 2; ++pers) {
                Pass t = ps;
                apply_leaf_tune(&t, {v, pers});
                PassArgs a = t.a;
                a.in = (char *)bin - ilo * (int64_t)eb;
                a.out = (char *)bout - olo * (int64_t)eb;
                hipError_t e = hipSuccess;
                for (int w = 0; w < 2 && e == hipSuccess; ++w)
                    e = launch_leaf(a, p->prob.prec, a.n, v, (int)t.grid, p->stream);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    continue;
                }
                const int reps = 5;
                (void)hipEventRecord(e0, p->stream);
                for (int r = 0; r < reps; ++r)
                    (void)launch_leaf(a, p->prob.prec, a.n, v, (int)t.grid, p->stream);
                (void)hipEventRecord(e1, p->stream);
                if (hipEventSynchronize(e1) != hipSuccess) {
                    rc = fail(MFFT_EHIP, "measurement failed");
                    break;
                }
                float ms = 0.f;
                (void)hipEventElapsedTime(&ms, e0, e1);
                if (ms < best) {
                    best = ms;
                    best_t = {v, pers};
                }
            }
            if (rc) break;
        }
        (void)hipStreamSynchronize(p->stream);
        (void)hipFree(bin);
        (void)hipFree(bout);
        if (rc) break;
        apply_leaf_tune(&ps, best_t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// "<structure>|<variants>": the structural choices ("n=...;n=...", or "-")
// and "i:v<variant>p<persistent>" for every pass that uses the leaf kernel
// (or "default").
std::string plan_choices(const PlanImpl *p)
{
    std::ostringstream s;
    bool first = true;
    for (auto &kv : p->overrides) {
        if (kv.second.empty()) continue;
        s << (first ? "" : ";") << choice_text(kv.first, kv.second);
        first = false;
    }
    if (first) s << "-";
    s << "|";
    first = true;
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const Pass &ps = p->passes[i];
        if (ps.kind != 0 || ps.kernel != 1) continue;
        s << (first ? "" : ";") << i << ":v" << ps.variant << "p" << ps.persistent;
        first = false;
    }
    if (first) s << "default";
    return s.str();
}

// Apply stored choices to a plan built with the same structural choices
// (the caller rebuilds the plan with the structural part first).
bool apply_choices(PlanImpl *p, const std::string &full)
{
    const size_t bar = full.find('|');
    const std::string text = bar == std::string::npos ? full : full.substr(bar + 1);
    if (text == "default") return true;
    std::vector<std::pair<size_t, LeafTune>> ch;
    std::istringstream s(text);
    std::string item;
    while (std::getline(s, item, ';')) {
        size_t i = 0;
        int v = 0, pe = 0;
        if (sscanf(item.c_str(), "%zu:v%dp%d", &i, &v, &pe) != 3) return false;
        if (i >= p->passes.size() || p->passes[i].kernel != 1) return false;
        if (v < 0 || v > 31 || pe < 0 || pe > 1) return false;
        ch.push_back({i, {v, pe}});
    }
    for (auto &c : ch) apply_leaf_tune(&p->passes[c.first], c.second);
    return true;
}

}  // namespace mfft
