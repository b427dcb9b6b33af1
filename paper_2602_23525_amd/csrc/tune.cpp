// Measure mode and wisdom (Section 4.3, "The FFTW planner"): build the plan
// for each applicable choice, time it, keep the fastest; choices can be saved
// and loaded later.  Each pass is optimized on its own, independently of the
// passes around it -- the dynamic-programming approximation the paper
// describes.  The tunable choice here is the variant of the specialized leaf
// kernel (prefetch, occupancy floor, non-temporal access) and its grid kind.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
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

// "i:v<variant>p<persistent>" for every pass that uses the leaf kernel.
std::string plan_choices(const PlanImpl *p)
{
    std::ostringstream s;
    bool first = true;
    for (size_t i = 0; i < p->passes.size(); ++i) {
        const Pass &ps = p->passes[i];
        if (ps.kind != 0 || ps.kernel != 1) continue;
        s << (first ? "" : ";") << i << ":v" << ps.variant << "p" << ps.persistent;
        first = false;
    }
    return first ? std::string("default") : s.str();
}

bool apply_choices(PlanImpl *p, const std::string &text)
{
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
