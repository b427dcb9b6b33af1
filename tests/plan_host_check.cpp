// The planner built for the host (device memory and kernel launches are stubs:
// tables get address ranges that are never dereferenced), then every planned
// pass checked against its tables.  For each table a pass reads -- gather and
// scatter indices, pre/post multipliers, the convolution spectrum, the
// two-level Cooley-Tukey twiddles, the stage twiddles of the generic kernel --
// the largest index any lane of any tile can form is computed from the pass
// descriptor the way the kernels form it, and must lie inside the allocation.
// Padding lines of a partial last tile (line index >= the vector length) take
// an in-range line's tables in both kernels; the check also reports how many
// passes would overrun a table if they did not (the lines the clamp protects).
// The generic kernel's LDS layouts between stages are simulated per pass:
// every read finds the element the previous step wrote there, inside the line.
//
// Usage:
//   plan_host_check bounds <prec> <n_lo> <n_hi> <batch> <primes|all|composite>
//     plans every 1-D length in [n_lo, n_hi] of that class, batch transforms
//     out of place, and checks them; prints one line per violation and a
//     summary "checked plans=P passes=S partial=Q guarded=G lds=L violations=V"
//     (L: passes whose LDS layouts were simulated).
//   plan_host_check plan <prec> <n> <batch>
//     prints the plan's pass list (as the library describes it).
//   plan_host_check cands <prec> <n_lo> <n_hi> <batch> [print]
//     every structural candidate measure mode would time for each length
//     (radix sequences, lines per tile, splits, Rader / Bluestein lengths),
//     planned with that choice and checked like the estimate's plan.
//   plan_host_check forced <prec> <n> <choice> <batch>
//     plans n with a structure choice forced on it ("r=16.8.8.8:b=2", the
//     wisdom grammar) and checks the plan.
//   plan_host_check steps <n> <R.R...>
//     plans one n-point transform with the radix sequence forced (Stockham
//     stages in execution order) and prints its stage descriptors, then the
//     plan as the list of DFT steps it executes, in breadth-first order (each
//     stage over the whole transform) and grouped depth-first (consecutive
//     steps that run under the same loop count nested in one loop).
//   plan_host_check random <count> <seed>
//     seeded random problems (rank 1-3 with vector loops, contiguous,
//     transposed or reversed strides, in place or not, both precisions, some
//     with aliasing outputs): canonicalized, planned when valid, checked.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "plan.h"

namespace mfft {

// ------------------------------------------------------------- launch stubs
hipError_t launch_real(const RealArgs &, int, hipStream_t) { return hipSuccess; }
hipError_t launch_gen_roots(void *, int, int64_t, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_pass(const PassArgs &, int, int, size_t, hipStream_t) { return hipSuccess; }
hipError_t launch_copy(const CopyArgs &, hipStream_t) { return hipSuccess; }
hipError_t launch_transpose_sq(const TransposeArgs &, hipStream_t) { return hipSuccess; }
hipError_t launch_permute_items(const PermuteArgs &, hipStream_t) { return hipSuccess; }
hipError_t launch_gen_stage_twiddles(void *, int, int, int, hipStream_t, bool, bool)
{
    return hipSuccess;
}
hipError_t launch_gen_tw4(void *, int64_t, void *, int64_t, int, int64_t, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_gen_chirp(void *, int64_t, hipStream_t) { return hipSuccess; }
hipError_t launch_gen_bluestein_v(void *, const void *, int64_t, int64_t, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_gen_rader(int32_t *, int32_t *, void *, int64_t, int64_t, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_convert_scale(void *, int, const void *, int64_t, double, hipStream_t)
{
    return hipSuccess;
}
hipError_t launch_leaf(const PassArgs &, int, int, int, int, hipStream_t) { return hipSuccess; }
// occupancy of the leaf kernel (only sizes persistent grids): one workgroup per CU
int leaf_blocks_per_cu(int, int, int) { return 1; }
// The device's answer modeled from the register use of the generic kernel
// variants (waves per SIMD: FP32 6, or 5 with twiddles; FP64 3, or 2; with 24
// elements per thread FP32 4, FP64 2), the LDS and 2048 threads per CU.
int pass_blocks_per_cu(int prec, int kind, int emax, int block, size_t lds)
{
    const int wps = emax > 16 ? (prec ? 2 : 4) : (prec ? (kind ? 2 : 3) : (kind ? 5 : 6));
    const int waves = (block + 63) / 64;
    int b = 4 * wps / waves;
    if (lds) b = std::min<int>(b, (int)((163840 - 256) / lds));
    b = std::min(b, 2048 / block);
    return b > 0 ? b : 1;
}

// The FP64 sub-plans that compute Rader and Bluestein spectra: no tables are
// computed on the host, so they plan nothing.
int plan_internal(mfft_plan *out, int, const mfft_iodim *, int, const mfft_iodim *, int, int, int,
                  hipStream_t, unsigned, const mfft_allocator *, int)
{
    *out = new mfft_plan_s();
    return MFFT_OK;
}

}  // namespace mfft

extern "C" int mfft_execute(mfft_plan, const void *, void *, void *) { return MFFT_OK; }
extern "C" int mfft_plan_destroy(mfft_plan p)
{
    delete p;
    return MFFT_OK;
}

using namespace mfft;

namespace mfft {
extern size_t g_lds_budget;
extern int g_num_cus;
}  // namespace mfft

// The device limits the library reads at its first plan on an MI355X
// (gfx950: 160 KB of LDS per workgroup less 256 bytes kept for the batched
// kernel's variables; 256 compute units), so that the host plans are the
// device's plans.
static void device_limits()
{
    g_lds_budget = 163840 - 256;
    g_num_cus = 256;
}

// Plan a 1-D problem on the host (canonicalize, then build the passes).
static int host_plan(PlanImpl *p, int prec, int64_t n, int64_t batch)
{
    mfft_iodim d{n, 1, 1};
    mfft_iodim v{batch, n, n};
    int rc = canonicalize(1, &d, batch > 1 ? 1 : 0, &v, 0, -1, prec, &p->prob);
    if (rc) return rc;
    return build_plan(p);
}

struct Checker {
    const PlanImpl *p;
    std::string name;
    int violations = 0, guarded = 0, lds_checked = 0;

    // bytes from ptr to the end of the table that holds it (-1: none)
    int64_t avail(const void *ptr) const
    {
        const uintptr_t x = (uintptr_t)ptr;
        for (const DeviceAlloc &t : p->tables) {
            const uintptr_t b = (uintptr_t)t.ptr;
            if (x >= b && x < b + t.bytes) return (int64_t)(b + t.bytes - x);
        }
        return -1;
    }

    // reads entries 0..max_index of `esize` bytes from ptr
    void need(const Pass &ps, const char *what, const void *ptr, int64_t max_index, int esize,
              int64_t unclamped)
    {
        if (!ptr) {
            std::printf("VIOLATION %s: %s table missing (%s)\n", name.c_str(), what, ps.desc.c_str());
            ++violations;
            return;
        }
        const int64_t a = avail(ptr);
        if (a < 0 || (max_index + 1) * esize > a) {
            std::printf("VIOLATION %s: %s index %lld, table holds %lld (%s)\n", name.c_str(), what,
                        (long long)max_index, (long long)(a / esize), ps.desc.c_str());
            ++violations;
        }
        if (unclamped > max_index && a >= 0 && (unclamped + 1) * esize > a) {
            std::printf("GUARDED %s: %s index %lld of a padding line, table holds %lld (%s)\n",
                        name.c_str(), what, (long long)unclamped, (long long)(a / esize),
                        ps.desc.c_str());
            ++guarded;
        }
    }

    // The generic kernel's LDS layouts of one pass (every pass has them: a
    // batch may run any pass in that kernel): each stage's butterfly b reads,
    // at b + (q >> rd_shift) + k*rd_stride, exactly the element b + k*nb the
    // tile load or the previous stage left there, writes element
    // q*Ns*R + j + k*Ns to a slot no other write of the stage takes, and every
    // slot lies inside the line's lds_stride; the last layout is unpadded (the
    // LDS store phase and a following transform read element i at i).
    void check_lds(const Pass &ps)
    {
        const PassArgs &a = ps.a;
        const int n = a.n, S = a.lds_stride;
        if (a.nst < 1 || n < 2) return;
        auto bad = [&](const char *what, int s, int b, int k) {
            std::printf("VIOLATION %s: LDS %s, stage %d butterfly %d element %d (%s)\n",
                        name.c_str(), what, s, b, k, ps.desc.c_str());
            ++violations;
        };
        if (n > S) return bad("line longer than its slots", -1, 0, 0);
        std::vector<int> cur(S, -1), nxt(S);
        for (int i = 0; i < n; ++i) cur[i] = i;   // the tile load: unpadded
        for (int s = 0; s < a.nst; ++s) {
            const StageDesc &sd = a.st[s];
            const int R = sd.R, Ns = sd.Ns, nb = n / R;
            if (sd.nb != nb || sd.rd_shift < 0 || sd.rd_shift > 31 || sd.wr_shift < 0 ||
                sd.wr_shift > 31)
                return bad("descriptor", s, 0, 0);
            std::fill(nxt.begin(), nxt.end(), -1);
            for (int b = 0; b < nb; ++b) {
                const int q = b / Ns, j = b - q * Ns;
                const int qd = (int)((((uint64_t)b * sd.magic >> 32) + (uint64_t)b) >> sd.shift);
                if (qd != q) return bad("quotient", s, b, 0);
                for (int k = 0; k < R; ++k) {
                    const int64_t ra = (int64_t)b + (q >> sd.rd_shift) + (int64_t)k * sd.rd_stride;
                    if (ra < 0 || ra >= S || cur[ra] != b + k * nb) return bad("read", s, b, k);
                    const int64_t wa = (int64_t)q * Ns * R + j + (q >> sd.wr_shift) + (int64_t)k * Ns;
                    if (wa < 0 || wa >= S || nxt[wa] != -1) return bad("write", s, b, k);
                    nxt[wa] = q * Ns * R + j + k * Ns;
                }
            }
            cur.swap(nxt);
        }
        for (int i = 0; i < n; ++i)
            if (cur[i] != i) return bad("last layout", a.nst, i, 0);
        ++lds_checked;
    }

    void check_pass(const Pass &ps)
    {
        if (ps.kind != 0) return;
        check_lds(ps);
        const PassArgs &a = ps.a;
        const int eb = ps.prec ? 16 : 8;
        const int64_t n = a.n;
        // line indices the kernels use for table lookups: the last line of the
        // vector loop at most; without the clamp, the last padding line
        const int64_t C = a.vn - 1;
        const int64_t Cu = a.ntiles_inner * a.bt - 1;
        const bool leaf = ps.kernel == 1;
        if (a.flags & PF_GATHER) need(ps, "gather", a.gather, a.li_lim - 1, 4, 0);
        if (a.flags & PF_PRE_MUL) need(ps, "pre", a.pre, a.li_lim - 1, eb, 0);
        if (a.flags & PF_SCATTER) need(ps, "scatter", a.scatter, a.lo_lim - 1, 4, 0);
        if (a.flags & PF_POST_MUL) {
            // leaf kernel, real-data split / combine: w_2n^k, k <= n/2
            const bool real = leaf && (a.flags & (PF_R2C | PF_C2R));
            need(ps, "post", a.post, real ? n / 2 : a.lo_lim - 1, eb, 0);
        }
        if (a.flags & PF_CONV)
            need(ps, "conv", a.conv, C * a.conv_c + (n - 1) * a.conv_k, eb,
                 Cu * a.conv_c + (n - 1) * a.conv_k);
        if (a.flags & PF_TW4) {
            // line c, element k: w_N^(c*k) from hi[e >> shift] * lo[e & mask];
            // FP32 data: e the lane's first exponent or its step (the rest by
            // products); FP64 data: e = c*k for every element
            int64_t step;
            if (ps.prec) step = n - 1;
            else if (leaf) step = n / 16;                     // threads per line
            else if (a.store_mode == kModeCol) step = a.tpt;  // lane stride of the store
            else step = a.st[a.nst - 1].Ns;                   // last stage's span
            const int64_t e = C * step, eu = Cu * step;
            if (e >= a.tw4_N) {
                std::printf("VIOLATION %s: twiddle exponent %lld >= N = %lld (%s)\n", name.c_str(),
                            (long long)e, (long long)a.tw4_N, ps.desc.c_str());
                ++violations;
            }
            need(ps, "tw4_hi", a.tw4_hi, e >> a.tw4_shift, 16, eu >> a.tw4_shift);
            need(ps, "tw4_lo", a.tw4_lo, a.tw4_mask, 16, 0);
        }
        // stage twiddles in the generic kernel's layout (every pass has them:
        // a batch may run any pass in that kernel): FP32 j-major, entry
        // tw_off + j*(R-1) + k-1 (j < Ns, 1 <= k < R); FP64 k-major, entry
        // tw_off + k*Ns + j (k < R); leaf-kernel passes also the k-major table
        for (int s = 0; s < a.nst; ++s) {
            const StageDesc &sd = a.st[s];
            if (sd.Ns > 1)
                need(ps, "stage", a.tw,
                     sd.tw_off + (int64_t)(ps.prec ? sd.R : sd.R - 1) * sd.Ns - 1, eb, 0);
        }
        if (leaf) {
            // laid out for the leaf kernel's own radix sequence (the one its
            // instantiations compile), whatever a.st holds
            int64_t total = 0, Ns = 1;
            for (int s = 0; s < leaf_radix_count(a.n); ++s) {
                total += Ns * leaf_radix_at(a.n, s);
                Ns *= leaf_radix_at(a.n, s);
            }
            if (Ns != a.n) {
                std::printf("VIOLATION %s: leaf radices do not multiply to n (%s)\n", name.c_str(),
                            ps.desc.c_str());
                ++violations;
            }
            need(ps, "stage (leaf layout)", a.tw_leaf, total - 1, eb, 0);
        }
        if (!leaf) {
            // per-transform Rader terms in scratch: entries 2*o, 2*o + 1
            if (a.flags & (PF_AUX_X0 | PF_AUX_A0 | PF_AUX_ADD)) {
                int64_t outer = 1;
                for (int d = 0; d < a.nouter; ++d) outer *= a.on[d];
                if (ps.aux_off < 0 || ps.aux_off + 2 * outer * eb > (int64_t)p->scratch_bytes) {
                    std::printf("VIOLATION %s: aux terms outside scratch (%s)\n", name.c_str(),
                                ps.desc.c_str());
                    ++violations;
                }
            }
        }
        // 32-bit logical indices of the table-driven loads and stores
        if ((a.flags & (PF_GATHER | PF_PRE_MUL)) && a.li_lim > INT32_MAX) ++violations;
        if ((a.flags & (PF_SCATTER | PF_POST_MUL)) && a.lo_lim > INT32_MAX) ++violations;
    }
};

// Random problem: lengths from a mix of small, smooth and prime values,
// strides of a contiguous array in a random axis order for each side, some
// reversed, sometimes a zero output stride (aliasing, to be refused).
static uint64_t rng_state;
static uint64_t rnd()
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static int random_problem(mfft_plan_s *pl, int *accepted)
{
    static const int64_t lens[] = {1, 2, 3, 4, 5, 7, 8, 12, 16, 17, 30, 64, 97, 100, 128,
                                   243, 256, 331, 1000, 1024, 2048, 4096, 6000, 8191};
    const int rank = 1 + (int)(rnd() % 3), vrank = (int)(rnd() % 3);
    const int tot = rank + vrank;
    int64_t n[6];
    int64_t elems = 1;
    for (int i = 0; i < tot; ++i) {
        n[i] = lens[rnd() % (sizeof(lens) / sizeof(lens[0]))];
        if (elems * n[i] > ((int64_t)1 << 24)) n[i] = 1 + (int64_t)(rnd() % 4);
        elems *= n[i];
    }
    int64_t is[6], os[6];
    for (int side = 0; side < 2; ++side) {
        int order[6];
        for (int i = 0; i < tot; ++i) order[i] = i;
        if (rnd() % 2)
            for (int i = tot - 1; i > 0; --i) std::swap(order[i], order[rnd() % (i + 1)]);
        int64_t st = 1;
        for (int k = tot - 1; k >= 0; --k) {
            const int i = order[k];
            (side ? os : is)[i] = (rnd() % 5 == 0) ? -st : st;
            st *= n[i];
        }
    }
    if (rnd() % 10 == 0) os[rnd() % tot] = 0;
    mfft_iodim d[3], v[3];
    for (int i = 0; i < rank; ++i) d[i] = {n[i], is[i], os[i]};
    for (int i = 0; i < vrank; ++i) v[i] = {n[rank + i], is[rank + i], os[rank + i]};
    const int inplace = (int)(rnd() % 3 == 0);
    const int prec = (int)(rnd() % 2);
    const int sign = rnd() % 2 ? 1 : -1;
    PlanImpl *p = &pl->impl;
    int rc = canonicalize(rank, d, vrank, v, inplace, sign, prec, &p->prob);
    if (rc) return rc == MFFT_EINVAL || rc == MFFT_ENOTSUP ? 0 : rc;
    *accepted = 1;
    rc = build_plan(p);
    return rc == MFFT_ENOTSUP ? 0 : rc;
}

static bool is_prime(int64_t n)
{
    if (n < 2) return false;
    for (int64_t f = 2; f * f <= n; ++f)
        if (n % f == 0) return false;
    return true;
}

int main(int argc, char **argv)
{
    device_limits();
    if (argc >= 7 && !std::strcmp(argv[1], "bounds")) {
        const int prec = std::atoi(argv[2]);
        const int64_t lo = std::atoll(argv[3]), hi = std::atoll(argv[4]), batch = std::atoll(argv[5]);
        const std::string cls = argv[6];
        int plans = 0, passes = 0, partial = 0, guarded = 0, violations = 0, failed = 0, lds = 0;
        for (int64_t n = lo; n <= hi; ++n) {
            const bool pr = is_prime(n);
            if (cls == "primes" && !pr) continue;
            if (cls == "composite" && pr) continue;
            mfft_plan_s pl;
            PlanImpl *p = &pl.impl;
            const int rc = host_plan(p, prec, n, batch);
            if (rc) {
                std::printf("PLAN FAILED n=%lld rc=%d\n", (long long)n, rc);
                ++failed;
                continue;
            }
            Checker ck{p, "n=" + std::to_string(n) + " c" + (prec ? "64" : "32")};
            for (const Pass &ps : p->passes) {
                ck.check_pass(ps);
                ++passes;
                if (ps.kind == 0 && ps.a.vn % ps.a.bt &&
                    (ps.a.flags & (PF_CONV | PF_TW4 | PF_PRE_MUL | PF_POST_MUL)))
                    ++partial;
            }
            violations += ck.violations;
            guarded += ck.guarded;
            lds += ck.lds_checked;
            ++plans;
        }
        std::printf("checked plans=%d passes=%d partial=%d guarded=%d lds=%d violations=%d failed=%d\n",
                    plans, passes, partial, guarded, lds, violations, failed);
        return violations || failed ? 1 : 0;
    }
    if (argc >= 5 && !std::strcmp(argv[1], "plan")) {
        mfft_plan_s pl;
        PlanImpl *p = &pl.impl;
        const int rc = host_plan(p, std::atoi(argv[2]), std::atoll(argv[3]), std::atoll(argv[4]));
        if (rc) {
            std::printf("PLAN FAILED rc=%d\n", rc);
            return 1;
        }
        for (const Pass &ps : p->passes)
            std::printf("%s vn=%lld bt=%d tiles=%lld\n", ps.desc.c_str(), (long long)ps.a.vn,
                        ps.a.bt, (long long)ps.a.ntiles);
        return 0;
    }
    if (argc >= 6 && !std::strcmp(argv[1], "cands")) {
        const int prec = std::atoi(argv[2]);
        const int64_t lo = std::atoll(argv[3]), hi = std::atoll(argv[4]), batch = std::atoll(argv[5]);
        const bool print = argc >= 7;
        int lengths = 0, cands = 0, planned = 0, violations = 0, failed = 0;
        for (int64_t n = lo; n <= hi; ++n) {
            mfft_plan_s base;
            if (host_plan(&base.impl, prec, n, batch)) continue;
            const auto cs = structure_candidates(&base.impl, n);
            ++lengths;
            for (size_t i = 0; i < cs.size(); ++i) {
                mfft_plan_s pl;
                PlanImpl *p = &pl.impl;
                if (!cs[i].empty()) p->overrides[n] = cs[i];
                ++cands;
                // the wisdom text of the choice reads back as the same choice
                int64_t n2 = 0;
                StructChoice c2;
                const std::string text = choice_text(n, cs[i]);
                if (!parse_choice(text, &n2, &c2) || n2 != n || choice_text(n2, c2) != text) {
                    std::printf("TEXT ROUND TRIP FAILED %s\n", text.c_str());
                    ++failed;
                }
                const int rc = host_plan(p, prec, n, batch);
                if (rc) {
                    std::printf("CANDIDATE FAILED n=%lld %s rc=%d\n", (long long)n,
                                choice_text(n, cs[i]).c_str(), rc);
                    ++failed;
                    continue;
                }
                ++planned;
                if (print) {
                    std::printf("%s\n", choice_text(n, cs[i]).c_str());
                    for (const Pass &ps : p->passes) std::printf("    %s\n", ps.desc.c_str());
                }
                Checker ck{p, "n=" + std::to_string(n) + " " + choice_text(n, cs[i])};
                for (const Pass &ps : p->passes) ck.check_pass(ps);
                violations += ck.violations;
            }
        }
        std::printf("checked lengths=%d candidates=%d planned=%d violations=%d failed=%d\n", lengths,
                    cands, planned, violations, failed);
        return violations || failed ? 1 : 0;
    }
    if (argc >= 6 && !std::strcmp(argv[1], "forced")) {
        // one length planned with a structure text forced on it (as wisdom
        // would), then checked like any plan
        const int prec = std::atoi(argv[2]);
        const int64_t n = std::atoll(argv[3]), batch = std::atoll(argv[5]);
        mfft_plan_s pl;
        PlanImpl *p = &pl.impl;
        int64_t n2 = 0;
        StructChoice c;
        if (!parse_choice("n=" + std::to_string(n) + ":" + argv[4], &n2, &c)) return 2;
        p->overrides[n] = c;
        if (host_plan(p, prec, n, batch)) {
            std::printf("PLAN FAILED\n");
            return 1;
        }
        Checker ck{p, "n=" + std::to_string(n) + " forced " + argv[4]};
        for (const Pass &ps : p->passes) {
            ck.check_pass(ps);
            std::printf("%s kernel=%d\n", ps.desc.c_str(), ps.kernel);
        }
        std::printf("checked passes=%d lds=%d violations=%d\n", (int)p->passes.size(), ck.lds_checked,
                    ck.violations);
        return ck.violations ? 1 : 0;
    }
    if (argc >= 4 && !std::strcmp(argv[1], "steps")) {
        const int64_t n = std::atoll(argv[2]);
        mfft_plan_s pl;
        PlanImpl *p = &pl.impl;
        int64_t n2 = 0;
        StructChoice c;
        if (!parse_choice("n=" + std::to_string(n) + ":r=" + argv[3], &n2, &c)) return 2;
        p->overrides[n] = c;
        if (host_plan(p, 1, n, 1) || p->passes.size() != 1 || p->passes[0].kernel != 0) return 1;
        const PassArgs &a = p->passes[0].a;
        struct Step {
            bool direct;
            int R;
            int64_t vec, loop;
        };
        std::vector<Step> steps;
        for (int st = 0; st < a.nst; ++st) {
            const StageDesc &sd = a.st[st];
            std::printf("stage R=%d Ns=%d nb=%d\n", sd.R, sd.Ns, sd.nb);
            if (st == 0) {
                // the first stage's butterflies have no twiddle: the direct
                // DFTs of the innermost step, vector of the next radix
                const int64_t v = a.nst > 1 ? a.st[1].R : 1;
                steps.push_back({true, sd.R, v, n / (sd.R * v)});
            } else {
                steps.push_back({false, sd.R, sd.Ns, n / ((int64_t)sd.R * sd.Ns)});
            }
        }
        auto one = [](const Step &t) {
            return std::string(t.direct ? "direct " : "twiddle ") + std::to_string(t.R) + " x" +
                   std::to_string(t.vec);
        };
        std::string br, de;
        for (size_t i = 0; i < steps.size(); ++i) {
            br += (i ? " ; " : "") + (steps[i].loop > 1 ? "loop " + std::to_string(steps[i].loop) +
                                                              " {" + one(steps[i]) + "}"
                                                        : one(steps[i]));
        }
        for (size_t i = 0; i < steps.size();) {
            size_t j = i;
            while (j + 1 < steps.size() && steps[j + 1].loop == steps[i].loop) ++j;
            std::string body;
            for (size_t k = i; k <= j; ++k) body += (k > i ? " ; " : "") + one(steps[k]);
            de += (i ? " ; " : "") +
                  (steps[i].loop > 1 ? "loop " + std::to_string(steps[i].loop) + " {" + body + "}" : body);
            i = j + 1;
        }
        std::printf("breadth: %s\ndepth: %s\n", br.c_str(), de.c_str());
        return 0;
    }
    if (argc >= 4 && !std::strcmp(argv[1], "random")) {
        const int count = std::atoi(argv[2]);
        rng_state = 0x9E3779B97F4A7C15ull ^ (uint64_t)std::atoll(argv[3]);
        int accepted = 0, planned = 0, violations = 0, failed = 0;
        for (int i = 0; i < count; ++i) {
            mfft_plan_s pl;
            int acc = 0;
            const int rc = random_problem(&pl, &acc);
            accepted += acc;
            if (rc) {
                std::printf("PLAN FAILED #%d rc=%d\n", i, rc);
                ++failed;
                continue;
            }
            if (!acc || pl.impl.passes.empty()) continue;
            ++planned;
            Checker ck{&pl.impl, "random #" + std::to_string(i)};
            for (const Pass &ps : pl.impl.passes) ck.check_pass(ps);
            violations += ck.violations;
        }
        std::printf("checked problems=%d accepted=%d planned=%d violations=%d failed=%d\n", count,
                    accepted, planned, violations, failed);
        return violations || failed ? 1 : 0;
    }
    std::fprintf(stderr, "usage: plan_host_check bounds|plan|random ...\n");
    return 2;
}
