// The planner: turns a canonical dft(N, V, I, O) into a list of GPU passes.
//
// Plan steps (Section 4.2), each realized as passes of the tile kernel:
//   - direct plan: a line of length n that fits one workgroup's LDS is one
//     pass (the leaf, a Stockham FFT held in LDS);
//   - Cooley-Tukey DIT step with radix r = n/m: pass A solves
//     dft({(m, r*is, os)}, V u {(r, is, m*os)}, I, O) and multiplies by the
//     twiddles w_n^(l2*k1) as it stores; pass B solves
//     dft({(r, m*os, m*os)}, copy-o(V) u {(m, os, os)}, O, O)  (four-step,
//     Section 3.1, used when n is larger than one leaf);
//   - vector loops become the launch grid (Section 4.2, "Plans for higher
//     vector ranks"); strided lines are loaded and stored through LDS tiles
//     across a unit-stride vector loop (vector recursion, Section 4.2.5);
//   - multi-dimensional transforms are one rank-1 step per dimension, the
//     first out of place, the rest in place on the output with copy-o strides
//     (Section 4.2 reduces rank > 1 to rank-1 problems);
//   - prime sizes: Rader's algorithm when p-1 factors into the supported
//     radices, Bluestein's chirp-z otherwise (Section 4.2, "Plans for prime
//     sizes"), each one kernel when the convolution fits a leaf; Bluestein's
//     length, and above 256 points the choice between the two, by estimated
//     cost; a composite length with one large prime factor as a Cooley-Tukey
//     step whose second pass is such a prime-size plan;
//   - rank 0: a copy (Section 4.2, "Rank-0 plans").
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <sstream>

#include "plan.h"

namespace mfft {

size_t g_lds_budget = 65536;   // bytes of LDS one workgroup may use
int g_num_cus = 256;           // compute units of the device


static int elem_bytes(int prec) { return prec ? 16 : 8; }
// workgroup size limit of the generic kernels (launch bounds in tile.h)
// (512 also for FP32 lines with 24 elements per thread: radices 17, 19, 23)
static int max_threads(int prec, int emax = 16) { return prec || emax > 16 ? 512 : 1024; }

// ------------------------------------------------------------ memory

void *dev_alloc(PlanImpl *p, size_t bytes)
{
    if (bytes == 0) return nullptr;
    void *ptr = nullptr;
    if (p->has_alloc && p->alloc.alloc) {
        ptr = p->alloc.alloc(bytes, (void *)p->stream, p->alloc.ctx);
    } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    return ptr;
}

void dev_free(PlanImpl *p, void *ptr, size_t bytes)
{
    (void)bytes;
    if (!ptr) return;
    if (p->has_alloc && p->alloc.free) p->alloc.free(ptr, (void *)p->stream, p->alloc.ctx);
    else (void)hipFree(ptr);
}

static void *table_alloc(PlanImpl *p, size_t bytes)
{
    void *ptr = dev_alloc(p, bytes);
    if (ptr) {
        p->tables.push_back({ptr, bytes});
        p->table_bytes += bytes;
    }
    return ptr;
}

// ------------------------------------------------------------ leaf shapes

struct Leaf {
    int n = 0;
    std::vector<int> rad;
    int emax = 16;
    int tpt = 0;
    int lds_stride = 0;
};

// Threads per line that a stage of radix R needs when a thread holds at most
// emax elements per stage.
static int stage_threads(int64_t n, int R, int emax)
{
    const int nbmax = emax / R;
    if (nbmax < 1) return INT32_MAX;
    return (int)((n / R + nbmax - 1) / nbmax);
}

// Elements per thread of a generic leaf of length n: 16, or 24 for lengths
// that need a radix 17, 19 or 23 (the kernel variant that holds them).
static int leaf_emax(int64_t n) { return is_smooth(n) ? 16 : 24; }

// Shortest LDS padding period of a generic leaf: 16 elements, or 64 for lines
// above 4096 points with 24 elements per thread (one line per tile: the
// saving lets two tiles share a CU, e.g. 10000 FP32 points in 81 KB rather
// than 85 KB).  Lines of 16 per thread keep 16: with 64, 12000 x 2048 FP32
// ran 178 -> 207 us from the bank conflicts of radix-16 stages.
static int pad_period_min(int64_t n, int emax) { return emax > 16 && n > 4096 ? 64 : 16; }

// 7-smooth lengths a generic leaf may also run with 24 elements per thread
// (plain and twiddled unit-stride lines; 512 threads hold them).
static bool wide_range(int64_t n) { return is_smooth(n) && n > 4096 && n <= 10240; }

// Radix sequence of a leaf of length n (smooth): the fewest stages over the
// radices the tile kernel compiles whose thread need fits max_tpt (each stage
// is one LDS exchange); among those, the smallest thread count, then larger
// radices first.  A dynamic program over the exponents of 2, 3, ..., 23
// (radices above 16 only with 24 elements per thread).
static bool radices_for(int64_t n, int emax, int max_tpt, std::vector<int> *r)
{
    if (n < 2 || !(emax >= 24 ? is_smooth23(n) : is_smooth(n))) return false;
    constexpr int NP = 9;
    static const int kRad[] = {23, 19, 17, 16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2};
    static const int kPrime[NP] = {2, 3, 5, 7, 11, 13, 17, 19, 23};
    using Ex = std::array<int, NP>;
    auto expo = [](int64_t v) {
        Ex e{};
        for (int i = 0; i < NP; ++i)
            while (v % kPrime[i] == 0) {
                v /= kPrime[i];
                ++e[i];
            }
        return e;
    };
    const Ex en = expo(n);
    size_t states = 1;
    for (int i = 0; i < NP; ++i) states *= (size_t)(en[i] + 1);
    auto index = [&](const Ex &e) {
        size_t x = 0;
        for (int i = 0; i < NP; ++i) x = x * (size_t)(en[i] + 1) + (size_t)e[i];
        return x;
    };
    struct Best {
        int stages = -1, need = 0, rad = 0;   // stages < 0: not computed; INT32_MAX: none
    };
    std::vector<Best> memo(states);
    std::vector<std::pair<int, Ex>> allowed;
    for (int R : kRad)
        if (stage_threads(n, R, emax) <= max_tpt) allowed.push_back({R, expo(R)});
    std::function<Best(const Ex &)> solve = [&](const Ex &a) -> Best {
        Best &m = memo[index(a)];
        if (m.stages >= 0) return m;
        Best best;
        bool done = true;
        for (int i = 0; i < NP; ++i) done &= a[i] == 0;
        best.stages = done ? 0 : INT32_MAX;
        if (!done) {
            for (const auto &re : allowed) {
                Ex rest = a;
                bool fits = true;
                for (int i = 0; i < NP; ++i) {
                    rest[i] -= re.second[i];
                    fits &= rest[i] >= 0;
                }
                if (!fits) continue;
                const Best sub = solve(rest);
                if (sub.stages == INT32_MAX) continue;
                const int st = sub.stages + 1;
                const int need = std::max(sub.need, stage_threads(n, re.first, emax));
                if (st < best.stages || (st == best.stages && need < best.need)) {
                    best.stages = st;
                    best.need = need;
                    best.rad = re.first;
                }
            }
        }
        memo[index(a)] = best;
        return best;
    };
    const Best top = solve(en);
    if (top.stages == INT32_MAX || top.stages > kMaxStages) return false;
    std::vector<int> rad;
    Ex a = en;
    for (;;) {
        bool done = true;
        for (int i = 0; i < NP; ++i) done &= a[i] == 0;
        if (done) break;
        const Best b = solve(a);
        rad.push_back(b.rad);
        const Ex e = expo(b.rad);
        for (int i = 0; i < NP; ++i) a[i] -= e[i];
    }
    std::sort(rad.begin(), rad.end(), std::greater<int>());
    *r = rad;
    return true;
}

static int line_lds_stride(int n, int emax)
{
    int s = n + (n - 1) / pad_period_min(n, emax) + 1;
    return s | 1;
}

// Dynamic LDS requested by scattering passes: at most two workgroups per CU.
constexpr size_t kScatterLdsBytes = 64 * 1024;

static size_t tile_lds_bytes(int n, int bt, int prec, int emax = 16)
{
    return ((size_t)bt * line_lds_stride(n, emax) + 2 * (size_t)bt) * elem_bytes(prec);
}

static bool leaf_shape_from(int64_t n, int emax, int max_tpt, const std::vector<int> &rad, Leaf *L);

static bool make_leaf_shape(int64_t n, int emax, int max_tpt, Leaf *L)
{
    if (n < 2 || n > (1 << 20)) return false;
    std::vector<int> rad;
    if (!radices_for(n, emax, max_tpt, &rad)) return false;
    return leaf_shape_from(n, emax, max_tpt, rad, L);
}

// The leaf shape of a given radix sequence (radices the tile kernel compiles,
// product n, thread need within max_tpt), or false.
static bool leaf_shape_from(int64_t n, int emax, int max_tpt, const std::vector<int> &rad, Leaf *L)
{
    if (n < 2 || n > (1 << 20) || rad.empty() || (int)rad.size() > kMaxStages) return false;
    int64_t prod = 1;
    for (int R : rad) {
        // radices 2..16 are compiled, and 17, 19, 23 with 24 elements per thread
        if (R < 2 || R > 23 || (R > 16 && (emax < 24 || (R != 17 && R != 19 && R != 23))))
            return false;
        if (stage_threads(n, R, emax) > max_tpt) return false;
        prod *= R;
    }
    if (prod != n) return false;
    int tpt = 1;
    for (int R : rad) tpt = std::max(tpt, stage_threads(n, R, emax));
    // the column loops unroll EMAX + 2 elements per thread
    tpt = std::max(tpt, (int)((n + emax + 1) / (emax + 2)));
    if (tpt > 1024) return false;
    L->n = (int)n;
    L->rad = rad;
    L->emax = emax;
    L->tpt = tpt;
    L->lds_stride = line_lds_stride((int)n, emax);
    return true;
}

// A plain unit-stride line of length n fits a leaf pass with 24 elements per
// thread.
static bool wide_leaf_fits(int64_t n, int prec)
{
    Leaf L;
    return wide_range(n) && make_leaf_shape(n, 24, max_threads(prec, 24), &L) &&
           tile_lds_bytes((int)n, 1, prec, 24) <= g_lds_budget;
}

// Estimate-mode choice of 24 elements per thread for a plain unit-stride
// line in wide_range: when 16 per thread has no one-pass shape, when 24 needs
// fewer stages (FP64 lines of 512 threads otherwise fall to radix 3), or when
// its half-size workgroups let more tiles share a CU without fewer resident
// threads (a 10000-point FP32 line: one 1000-thread workgroup per CU, or two
// of 500).  Measured on MI355X, 16 -> 24: 10000 x 2048 FP32 127 -> 103 us,
// 8000 x 2048 107 -> 95 us, 6561 x 2048 FP64 228 -> 161 us, 8000 x 1024 FP64
// 164 -> 98 us (two passes -> one); 6561 x 4096 FP32 139 -> 158 us (two
// workgroups of 729 threads per CU against two of 365) keeps 16.
static bool prefer_wide(int64_t n, int prec, int kind)
{
    if (!wide_leaf_fits(n, prec)) return false;
    Leaf a, w;
    make_leaf_shape(n, 24, max_threads(prec, 24), &w);
    if (!make_leaf_shape(n, 16, max_threads(prec, 16), &a) ||
        tile_lds_bytes((int)n, 1, prec) > g_lds_budget)
        return true;
    if (w.rad.size() < a.rad.size()) return true;
    const int o16 = pass_blocks_per_cu(prec, kind, 16, a.tpt, tile_lds_bytes((int)n, 1, prec));
    const int o24 = pass_blocks_per_cu(prec, kind, 24, w.tpt, tile_lds_bytes((int)n, 1, prec, 24));
    return o24 > o16 && (int64_t)o24 * w.tpt >= (int64_t)o16 * a.tpt;
}

// A line of length n fits a leaf pass with at least `bt` lines per tile.
static bool leaf_fits(int64_t n, int prec, int bt)
{
    Leaf L;
    const int mt = max_threads(prec, leaf_emax(n));
    if (!make_leaf_shape(n, leaf_emax(n), mt / bt, &L)) return false;
    return tile_lds_bytes((int)n, bt, prec, L.emax) <= g_lds_budget && bt * L.tpt <= mt;
}

// Stage twiddle tables of a leaf: stage s holds w_(Ns*R)^(j*k) for j < Ns.
// k-major: 0 <= k < R at [off_s + k*Ns + j] (the lanes of a wave, which work
// on consecutive j, read consecutive entries); j-major: 1 <= k < R at
// [off_s + j*(R-1) + k-1] (a butterfly's twiddles are consecutive: one address
// and immediate offsets).  The generic tile kernel reads FP32 tables j-major
// (measured on MI355X, FP32: 1000 x 16384 83.6 -> 80.3 us, 6561 x 4096 213 ->
// 199 us) and FP64 tables k-major (j-major 1000 x 8192 FP64: 70.7 -> 82.9 us:
// rows of 16-byte twiddles spread a wave's load over too many cache lines),
// at tw + st[s].tw_off; every pass has that table, since a batch may run any
// pass in the generic kernel.  A pass planned for the specialized leaf kernel
// also gets the k-major table it reads, in tw_leaf.
static int stage_table(PlanImpl *p, const Leaf &L, bool jmajor, std::map<std::string, void *> *cache,
                       const void **out)
{
    std::ostringstream key;
    key << p->prob.prec << ":" << L.n << (jmajor ? "j" : "k");
    for (int R : L.rad) key << "," << R;
    auto it = cache->find(key.str());
    if (it != cache->end()) {
        *out = it->second;
        return MFFT_OK;
    }
    int64_t total = 0;
    for (int64_t s = 0, Ns = 1; s < (int64_t)L.rad.size(); Ns *= L.rad[s], ++s)
        total += Ns * (jmajor ? L.rad[s] - 1 : L.rad[s]);
    const size_t eb = elem_bytes(p->prob.prec);
    void *tw = table_alloc(p, (size_t)std::max<int64_t>(total, 1) * eb);
    if (!tw) return fail(MFFT_ENOMEM, "twiddle table allocation failed");
    int64_t off = 0;
    for (int64_t s = 0, Ns = 1; s < (int64_t)L.rad.size(); Ns *= L.rad[s], ++s) {
        const int R = L.rad[s];
        if (Ns > 1) {
            hipError_t e = launch_gen_stage_twiddles((char *)tw + (size_t)off * eb, p->prob.prec,
                                                     (int)Ns, R, p->stream,
                                                     (p->flags & MFFT_FP32_TWIDDLES) != 0, jmajor);
            if (e != hipSuccess)
                return fail(MFFT_EHIP, std::string("twiddle kernel: ") + hipGetErrorString(e));
        }
        off += Ns * (jmajor ? R - 1 : R);
    }
    (*cache)[key.str()] = tw;
    *out = tw;
    return MFFT_OK;
}

// Bank-conflict cycles of one LDS access by a wave whose lane l touches
// complex element addr[l] (eb bytes; negative: lane idle), summed over two
// models of the LDS: 32 and 64 banks of 4 bytes, lanes served in groups that
// cover the banks once.
static int lds_access_cycles(const int (&addr)[64], int eb)
{
    int total = 0;
    for (int banks : {32, 64}) {
        const int group = std::max(1, banks * 4 / eb), words = eb / 4;
        for (int l0 = 0; l0 < 64; l0 += group) {
            int cnt[64] = {};
            int worst = 0;
            for (int l = l0; l < l0 + group && l < 64; ++l) {
                if (addr[l] < 0) continue;
                for (int w = 0; w < words; ++w) {
                    const int bank = (int)(((int64_t)addr[l] * words + w) % banks);
                    worst = std::max(worst, ++cnt[bank]);
                }
            }
            total += worst;
        }
    }
    return total;
}

// LDS layouts of a generic leaf's stages (StageDesc::rd_stride, rd_shift,
// wr_shift): for each stage boundary, the padding period G*2^sh (G = Ns*R of
// the writing stage) or none, among those of at least pad_period_min(n, emax)
// elements (a line then never needs more than line_lds_stride(n, emax) slots) that
// divide the next
// stage's butterfly count (its reads stay affine), with the fewest modeled
// bank-conflict cycles over the first wave's writes and the next stage's
// reads; ties go to no padding, then to the longer period.
void lds_layouts(int n, int nst, int tpt, int lds_stride, int emax, int eb, StageDesc *st)
{
    const int pmin = pad_period_min(n, emax);
    constexpr int kNone = 31;
    auto lane_cost = [&](int s, int sh, bool write) {
        const StageDesc &sd = st[s];
        const int R = sd.R, Ns = sd.Ns, G = Ns * R, nbs = n / R;
        int cost = 0;
        for (int i = 0; i < emax / R; ++i)
            for (int k = 0; k < R; ++k) {
                int addr[64];
                for (int l = 0; l < 64; ++l) {
                    const int tr = l / tpt, t = l % tpt, b = t + i * tpt;
                    const int q = b / Ns, j = b - q * Ns;
                    addr[l] = b >= nbs ? -1
                                       : tr * lds_stride +
                                             (write ? q * G + j + (sh == kNone ? 0 : q >> sh) + k * Ns
                                                    : b + (sh == kNone ? 0 : q >> sh) + k * sd.rd_stride);
                }
                cost += lds_access_cycles(addr, eb);
            }
        return cost;
    };
    st[0].rd_shift = kNone;
    st[0].rd_stride = n / st[0].R;
    for (int s = 0; s < nst; ++s) {
        StageDesc &sd = st[s];
        sd.wr_shift = kNone;
        if (s + 1 == nst) break;   // the last layout is unpadded
        StageDesc &nx = st[s + 1];
        const int G = sd.Ns * sd.R, nbn = n / nx.R;
        int best_cost = INT32_MAX, best = kNone;
        for (int sh = kNone; sh >= 0; sh = sh == kNone ? 20 : sh - 1) {
            int rstride = nbn;
            if (sh != kNone) {
                const int64_t per = (int64_t)G << sh;
                if (per < pmin || per > nbn || nbn % per != 0) continue;
                rstride = nbn + (int)(nbn / per);
            }
            nx.rd_stride = rstride;
            const int cost = lane_cost(s, sh, true) + lane_cost(s + 1, sh, false);
            if (cost < best_cost) {
                best_cost = cost;
                best = sh;
            }
        }
        sd.wr_shift = (int16_t)best;
        nx.rd_shift = (int16_t)best;
        nx.rd_stride = best == kNone ? nbn : nbn + nbn / (G << best);
    }
}

static int fill_leaf(PlanImpl *p, const Leaf &L, PassArgs *a,
                     std::map<std::string, void *> *cache, bool leaf_kernel)
{
    const bool jmajor = p->prob.prec == 0;   // the generic kernel's layout
    int64_t off = 0;
    int Ns = 1;
    a->n = L.n;
    a->nst = (int)L.rad.size();
    a->tpt = L.tpt;
    a->lds_stride = L.lds_stride;
    for (size_t s = 0; s < L.rad.size(); ++s) {
        StageDesc &sd = a->st[s];
        sd.R = L.rad[s];
        sd.Ns = Ns;
        div_magic((uint32_t)Ns, &sd.magic, &sd.shift);
        sd.tw_off = (int32_t)off;
        sd.nb = L.n / sd.R;
        off += (int64_t)Ns * (jmajor ? sd.R - 1 : sd.R);
        Ns *= sd.R;
    }
    lds_layouts(L.n, a->nst, L.tpt, L.lds_stride, L.emax, (int)elem_bytes(p->prob.prec), a->st);
    int rc = stage_table(p, L, jmajor, cache, &a->tw);
    if (rc == MFFT_OK && leaf_kernel) {
        // the leaf kernel's own radix sequence (its table layout), which a
        // measured or imported structure for this length does not change
        Leaf Lk = L;
        Lk.rad.clear();
        for (int i = 0; i < leaf_radix_count(L.n); ++i) Lk.rad.push_back(leaf_radix_at(L.n, i));
        rc = stage_table(p, Lk, false, cache, &a->tw_leaf);
    }
    return rc;
}

// ------------------------------------------------------------ pass building

// ------------------------------------------------------------ leaf variants

// Estimate-mode choice of the leaf kernel variant (measured on MI355X over
// batched unit-stride transforms of 64 to 4096 points, both precisions, 16 MB
// to 512 MB per buffer, executed repeatedly on the same buffers): one tile
// per workgroup; stores non-temporal, loads too once a buffer exceeds the
// 256 MB last-level cache (a smaller input is usually still there from the
// kernel that wrote it, and cached loads then run 5-15% faster).  A line
// whose tile fills the LDS of a CU alone (16384 points FP32, 8192 FP64) runs
// on a persistent grid of one workgroup per CU: launching a new workgroup
// after each tile left the CU idle in between (16384 x 4096 FP32: 251 ->
// 225 us; 8192 x 4096 FP64: 232 -> 218 us).
LeafTune leaf_default(int prec, int n, double in_bytes)
{
    const bool fills_cu = (int64_t)n * elem_bytes(prec) >= 128 * 1024;
    return {in_bytes > 256.0 * 1024 * 1024 ? 24 : 8, fills_cu ? 1 : 0};
}

void apply_leaf_tune(Pass *ps, const LeafTune &t)
{
    ps->variant = t.variant;
    ps->persistent = t.persistent;
    ps->grid = ps->a.ntiles;
    if (t.persistent) {
        const int64_t resident =
            (int64_t)leaf_blocks_per_cu(ps->prec, ps->a.n, t.variant) * g_num_cus;
        ps->grid = std::min<int64_t>(ps->a.ntiles, std::max<int64_t>(resident, 1));
    }
}

struct LineSpec {
    Dim line;                  // (n, is, os) of the line
    std::vector<Dim> V;        // vector loops
    int inner = -1;            // forced index of the tiled loop in V (-1 = choose)
    int src = BUF_IN, dst = BUF_OUT;
    int64_t src_off = 0, dst_off = 0;
    uint32_t flags = 0;
    int64_t li_c = 0, li_l = 1, li_lim = -1;   // -1: n
    int64_t lo_c = 0, lo_k = 1, lo_lim = -1;
    int64_t tw4_N = 0;
    const void *pre = nullptr, *post = nullptr, *conv = nullptr;
    // the spectrum as a column tile reads it (entry c*conv_cols_c + k*conv_cols_k
    // for element k of line c), when the pass may run in the leaf kernel
    const void *conv_cols = nullptr;
    int64_t conv_cols_c = 0, conv_cols_k = 0;
    const int32_t *gather = nullptr, *scatter = nullptr;
    int64_t aux_off = -1;
    int64_t conv_n = 0;        // leaf length when it differs from line.n (Bluestein / Rader)
    int64_t conv_c = 0, conv_k = 1;   // convolution table index c*conv_c + k*conv_k
    std::string what;
};

struct Builder {
    PlanImpl *p;
    std::map<std::string, void *> twcache;
    std::map<int64_t, std::pair<void *, void *>> tw4cache;
    int64_t scratch_top = 0;   // bytes
    int64_t scratch_hi = 0;

    int64_t scratch_take(int64_t bytes)
    {
        int64_t off = (scratch_top + 255) / 256 * 256;
        scratch_top = off + bytes;
        scratch_hi = std::max(scratch_hi, scratch_top);
        return off;
    }
};

static int ilog2(int x)
{
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}

static int tw4_tables(Builder &b, int64_t N, PassArgs *a)
{
    int shift = 0;
    while (((int64_t)1 << (2 * shift)) < N) ++shift;     // 2^shift ~ sqrt(N)
    const int64_t nlo = (int64_t)1 << shift;
    const int64_t nhi = (N + nlo - 1) / nlo;
    auto it = b.tw4cache.find(N);
    void *hi, *lo;
    if (it != b.tw4cache.end()) {
        hi = it->second.first;
        lo = it->second.second;
    } else {
        hi = table_alloc(b.p, (size_t)nhi * 16);
        lo = table_alloc(b.p, (size_t)nlo * 16);
        if (!hi || !lo) return fail(MFFT_ENOMEM, "twiddle table allocation failed");
        hipError_t e = launch_gen_tw4(hi, nhi, lo, nlo, shift, N, b.p->stream);
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("tw4 kernel: ") + hipGetErrorString(e));
        b.tw4cache[N] = {hi, lo};
    }
    a->tw4_hi = hi;
    a->tw4_lo = lo;
    a->tw4_N = N;
    a->tw4_shift = shift;
    a->tw4_mask = (int32_t)(nlo - 1);
    return MFFT_OK;
}

static std::string dims_str(const Dim &d) {
    std::ostringstream s;
    s << "(" << d.n << "," << d.is << "," << d.os << ")";
    return s.str();
}

// The leaf kernel takes a pass with column tiles when its lines are plain
// (at most conjugation and the Cooley-Tukey twiddle on store), of a supported
// length, adjacent (unit vector stride) on each column side and of unit
// element stride on a row side.
static bool leaf_col_fits(const LineSpec &ls, const PassArgs &a, const Dim &in_dim, int prec,
                          int64_t n)
{
    const bool cin = a.load_mode == kModeCol, cout = a.store_mode == kModeCol;
    if (!cin && !cout) return false;
    const bool xp = cin != cout;
    // Bluestein's outer passes: the chirp product (and zero padding) on the
    // loads of a columns-in tile, the chirp product (and truncation) on the
    // stores of a columns-out tile
    const uint32_t allowed = PF_CONJ_IN | PF_CONJ_OUT | PF_TW4 |
                             (xp && cin ? PF_PRE_MUL : 0) | (xp && cout ? PF_POST_MUL | PF_CONJ_A : 0) |
                             (!xp && ls.conv_cols ? PF_CONV : 0);
    if ((ls.flags & ~allowed) || ls.conv_n) return false;
    if (!leaf_col_supported(prec, n, xp)) return false;
    if (cin ? in_dim.is != 1 : ls.line.is != 1) return false;
    if (cout ? in_dim.os != 1 : ls.line.os != 1) return false;
    return true;
}

// Lines per tile of a row tile (lanes along the lines, so any count works):
// the workgroup of bt * tpt threads rounds up to the 256-, 512- or 1024-thread
// class that batched launches use, with a tile of at most 64 KB of LDS (two or
// more workgroups per CU) and no more lines than the vector loop has.  Among
// the classes, the one that keeps the most working lanes resident on a CU (bt
// * tpt times the workgroups per CU that registers and LDS allow); ties go to
// the smaller.  Filling the class alone chose 73 lines of 98 points (511 of
// 512 threads, 62 KB, two workgroups per CU) where 36 lines (252 of 256, five
// per CU) run 98 x 65536 FP32 in 31 rather than 33 us (MI355X); powers of two
// alone left up to a quarter of the lanes idle (200 of 256 threads for
// 1000-point lines).
int row_lines_per_tile(int n, int tpt, int prec, int64_t lines, int emax)
{
    const int e = emax ? emax : leaf_emax(n);
    const int mt = max_threads(prec, e);
    int best = 1;
    int64_t best_live = -1;
    for (int cls = 256; cls <= mt; cls *= 2) {
        int bt = std::max(1, cls / tpt);
        while (bt > 1 && tile_lds_bytes(n, bt, prec, e) > 65536) --bt;
        while (bt > 1 && tile_lds_bytes(n, bt, prec, e) > g_lds_budget) --bt;
        if (lines > 0) bt = (int)std::max<int64_t>(1, std::min<int64_t>(bt, lines));
        int block = 256;
        while (block < bt * tpt) block *= 2;
        const int64_t live =
            (int64_t)bt * tpt * pass_blocks_per_cu(prec, 0, e, block, tile_lds_bytes(n, bt, prec, e));
        if (live > best_live) {
            best_live = live;
            best = bt;
        }
    }
    return best;
}

static const StructChoice *choice_for(const PlanImpl *p, int64_t n)
{
    auto it = p->overrides.find(n);
    return it == p->overrides.end() ? nullptr : &it->second;
}

static int add_line_pass(Builder &b, const LineSpec &ls)
{
    PlanImpl *p = b.p;
    const int prec = p->prob.prec;
    const int64_t n = ls.conv_n ? ls.conv_n : ls.line.n;
    const StructChoice *ch = choice_for(p, n);
    Pass ps;
    PassArgs &a = ps.a;
    ps.prec = prec;
    // choose the tiled (inner) vector loop
    std::vector<Dim> V = ls.V;
    int inner = ls.inner;
    const bool row_in = std::llabs(ls.line.is) == 1 || (ls.flags & PF_GATHER);
    const bool row_out = std::llabs(ls.line.os) == 1 || (ls.flags & PF_SCATTER);
    if (inner < 0 && !V.empty()) {
        int best = -1;
        int64_t best_score = INT64_MIN;
        for (size_t i = 0; i < V.size(); ++i) {
            int64_t sc = 0;
            if (!row_in && std::llabs(V[i].is) == 1) sc += 4;
            if (!row_out && std::llabs(V[i].os) == 1) sc += 4;
            if (row_in && row_out) sc -= std::llabs(V[i].is);   // any loop; prefer small stride
            sc = sc * 64 + std::min<int64_t>(V[i].n, 63);
            if (sc > best_score) {
                best_score = sc;
                best = (int)i;
            }
        }
        inner = best;
    }
    Dim in_dim{1, 0, 0};
    if (inner >= 0) {
        in_dim = V[inner];
        V.erase(V.begin() + inner);
    }
    if ((int)V.size() > kMaxOuter) return fail(MFFT_ENOTSUP, "too many vector loops for one pass");
    a.vn = in_dim.n;
    a.vis = in_dim.is;
    a.vos = in_dim.os;
    a.nouter = (int)V.size();
    int64_t nouter_total = 1;
    for (size_t i = 0; i < V.size(); ++i) {
        a.on[i] = V[i].n;
        a.ois[i] = V[i].is;
        a.oos[i] = V[i].os;
        nouter_total *= V[i].n;
    }
    a.load_mode = (!row_in && std::llabs(in_dim.is) < std::llabs(ls.line.is) && in_dim.n > 1)
                      ? kModeCol : kModeRow;
    a.store_mode = (!row_out && std::llabs(in_dim.os) < std::llabs(ls.line.os) && in_dim.n > 1)
                       ? kModeCol : kModeRow;
    if ((ls.flags & PF_GATHER) && a.load_mode == kModeCol) a.load_mode = kModeRow;

    // lines per tile: column phases want >= 128 B runs; row tiles aim at
    // 256-thread workgroups.  Both bounded by the LDS budget.
    const bool col = a.load_mode == kModeCol || a.store_mode == kModeCol;
    const int bt_floor = col ? (prec ? 4 : 8) : 1;
    // elements per thread: 24 for radices 17, 19, 23; for plain and twiddled
    // unit-stride row lines in wide_range as measured or estimated; else 16
    const bool plain_tw = !(ls.flags & ~(PF_CONJ_IN | PF_CONJ_OUT | PF_TW4 | PF_XCD));
    int emax = leaf_emax(n);
    if (emax > 16 && !plain_tw)
        return fail(MFFT_ENOTSUP, "radices above 16 only in plain or twiddled lines");
    if (emax == 16 && plain_tw && !col && ls.line.is == 1 && ls.line.os == 1 && wide_range(n)) {
        const int kind = (ls.flags & PF_TW4) ? 1 : 0;
        if (ch && ch->emax) {
            if (ch->emax == 24 && wide_leaf_fits(n, prec)) emax = 24;
        } else if (prefer_wide(n, prec, kind)) {
            emax = 24;
        }
    }
    const int mt = max_threads(prec, emax);
    Leaf L;
    if (!make_leaf_shape(n, emax, mt / bt_floor, &L) && !make_leaf_shape(n, emax, mt, &L))
        return fail(MFFT_ENOTSUP, "no leaf shape for n");
    if (ch && !ch->rad.empty()) {
        // a measured radix sequence (if it fits this pass's thread budget)
        Leaf Lc;
        if (leaf_shape_from(n, emax, mt / bt_floor, ch->rad, &Lc)) L = Lc;
    }
    ps.emax = L.emax;
    a.n = L.n;   // the stage tables are filled once the kernel is chosen
    int rc = MFFT_OK;
    // Prefer tiles of at most 64 KB (several workgroups per CU); column tiles
    // may grow to the full LDS rather than drop below 64-byte runs.
    int bt;
    if (col) {
        // 16 lines: 128-byte runs FP32, 256-byte FP64 (FP64 against 8 lines:
        // 14175 x 512 151 -> 140 us, 20000 x 128 64 -> 62 us, MI355X)
        bt = 16;
        while (bt > bt_floor && (tile_lds_bytes(L.n, bt, prec, L.emax) > 65536 || bt * L.tpt > mt)) bt >>= 1;
        while (bt > 1 && (tile_lds_bytes(L.n, bt, prec, L.emax) > g_lds_budget || bt * L.tpt > mt)) bt >>= 1;
        while (bt > 1 && bt / 2 >= in_dim.n) bt >>= 1;   // no wider than the loop
    } else {
        bt = row_lines_per_tile(L.n, L.tpt, prec, in_dim.n, L.emax);
        if (ch && ch->bt > 0 && ch->bt * L.tpt <= mt &&
            tile_lds_bytes(L.n, ch->bt, prec, L.emax) <= g_lds_budget)
            bt = (int)std::max<int64_t>(1, std::min<int64_t>(ch->bt, in_dim.n));
    }
    if (tile_lds_bytes(L.n, bt, prec, L.emax) > g_lds_budget || bt * L.tpt > mt)
        return fail(MFFT_ENOTSUP, "leaf does not fit the LDS budget");
    a.bt = bt;
    a.bt_log2 = ilog2(bt);
    a.ntiles_inner = (a.vn + bt - 1) / bt;
    a.ntiles = a.ntiles_inner * nouter_total;
    ps.lds_bytes = tile_lds_bytes(L.n, bt, prec, L.emax);
    if ((ls.flags & PF_SCATTER) && (ls.flags & PF_XCD)) {
        // A scattering pass fills each cache line of its output from many
        // tiles; lines written back before they are full cost a partial
        // write each (measured: 5x the output bytes at 4 workgroups per CU).
        // Two workgroups per CU keep the partially written output of the
        // tiles in flight on one XCD near 2 MB, within its 4 MB L2.
        ps.lds_bytes = std::max<size_t>(ps.lds_bytes, kScatterLdsBytes);
    }

    a.is = ls.line.is;
    a.os = ls.line.os;
    a.flags = ls.flags;
    // Plain stores stream past the caches when one store instruction of a
    // wave covers whole 128-byte lines: unit-stride runs of the lanes of one
    // line (row stores) or of the tile's lines (column stores); shorter runs
    // keep cached stores, which the L2 merges into whole lines.  Measured on
    // MI355X (FP32, same box): long runs gain 2-5% (1000 x 16384 78.5 ->
    // 75.7 us, 3000 x 8192 133 -> 127 us, 14175 x 512 51.5 -> 48.7 us); runs
    // of 16-96 bytes (30, 60, 98, 144 points per line) differ by less than
    // the 2-3% run-to-run spread either way.
    {
        const int64_t run = a.store_mode == kModeCol ? (std::llabs(in_dim.os) == 1 ? bt : 1)
                                                     : (std::llabs(a.os) == 1 ? std::min(L.tpt, 64) : 1);
        if (run * (int64_t)elem_bytes(prec) >= 128) a.flags |= PF_NT_OUT;
    }
    a.li_c = ls.li_c;
    a.li_l = ls.li_l;
    a.li_lim = ls.li_lim < 0 ? n : ls.li_lim;
    a.lo_c = ls.lo_c;
    a.lo_k = ls.lo_k;
    a.lo_lim = ls.lo_lim < 0 ? n : ls.lo_lim;
    a.pre = ls.pre;
    a.post = ls.post;
    a.conv = ls.conv;
    a.conv_c = ls.conv_c;
    a.conv_k = ls.conv_k;
    a.gather = ls.gather;
    a.scatter = ls.scatter;
    if (ls.flags & PF_TW4) {
        rc = tw4_tables(b, ls.tw4_N, &a);
        if (rc) return rc;
    }
    // unit-stride plain lines of a power-of-two length: the specialized leaf
    // kernel; so too Bluestein in one tile over a power-of-two convolution
    const uint32_t plain = PF_CONJ_IN | PF_CONJ_OUT;
    const uint32_t blue1 = PF_CONV | PF_PRE_MUL | PF_POST_MUL | PF_CONJ_A;
    const bool leaf_blue = ls.conv_n && (ls.flags & ~plain) == blue1 && ls.li_c == 0 &&
                           ls.li_l == 1 && ls.lo_c == 0 && ls.lo_k == 1 && ls.conv_c == 0 &&
                           ls.conv_k == 1;
    if ((leaf_blue || (!(ls.flags & ~plain) && !ls.conv_n)) && ls.line.is == 1 &&
        ls.line.os == 1 && a.load_mode == kModeRow && a.store_mode == kModeRow &&
        leaf_supported(prec, n)) {
        ps.kernel = 1;
        a.bt = leaf_lines_per_tile(prec, (int)n);
        a.bt_log2 = ilog2(a.bt);
        a.ntiles_inner = (a.vn + a.bt - 1) / a.bt;
        a.ntiles = a.ntiles_inner * nouter_total;
        ps.lds_bytes = 0;
        LeafTune t = leaf_default(prec, (int)n, (double)a.vn * nouter_total * n * elem_bytes(prec));
        apply_leaf_tune(&ps, t);
    } else if (leaf_col_fits(ls, a, in_dim, prec, n)) {
        // adjacent lines with strided elements (columns of a row-major array)
        // on one side or both: the leaf kernel with column tiles
        const bool cin = a.load_mode == kModeCol, cout = a.store_mode == kModeCol;
        ps.kernel = 1;
        a.flags |= cin && cout ? PF_LEAF_COL : (cin ? PF_LEAF_CR : PF_LEAF_RC);
        if (ls.flags & PF_CONV) {
            a.conv = ls.conv_cols;
            a.conv_c = ls.conv_cols_c;
            a.conv_k = ls.conv_cols_k;
        }
        a.bt = leaf_col_lines_per_tile(prec, (int)n);
        a.bt_log2 = ilog2(a.bt);
        a.ntiles_inner = (a.vn + a.bt - 1) / a.bt;
        a.ntiles = a.ntiles_inner * nouter_total;
        ps.lds_bytes = 0;
        apply_leaf_tune(&ps, {24, 0});   // the one configuration of column tiles
    }
    rc = fill_leaf(p, L, &a, &b.twcache, ps.kernel == 1);
    if (rc) return rc;
    ps.src = ls.src;
    ps.dst = ls.dst;
    ps.src_off = ls.src_off;
    ps.dst_off = ls.dst_off;
    ps.aux_off = ls.aux_off;
    const int64_t lines = a.vn * nouter_total;
    const int64_t nin = std::min<int64_t>(a.li_lim, n), nout = std::min<int64_t>(a.lo_lim, n);
    ps.bytes = (double)lines * (double)(nin + nout) * elem_bytes(prec);
    if (ls.flags & (PF_CONV)) ps.bytes = (double)lines * (double)(ls.line.n * 2) * elem_bytes(prec);
    std::ostringstream d;
    d << ls.what << " n=" << n << " rad=";
    for (size_t i = 0; i < L.rad.size(); ++i) d << (i ? "x" : "") << L.rad[i];
    d << " tpt=" << L.tpt << " bt=" << a.bt << " " << (a.load_mode ? "C" : "R")
      << (a.store_mode ? "C" : "R") << " line=" << dims_str(ls.line) << " inner=" << dims_str(in_dim)
      << " tiles=" << a.ntiles;
    ps.desc = d.str();
    p->passes.push_back(ps);
    return MFFT_OK;
}

// ------------------------------------------------------------ rank-1 algorithms

static std::vector<Dim> copy_o(const std::vector<Dim> &V)
{
    std::vector<Dim> r;
    for (const Dim &d : V) r.push_back({d.n, d.os, d.os});
    return r;
}

// Packed layout of the vector loops in a scratch buffer whose transforms are
// `per` elements apart: returns V with input strides replaced (which=0) or
// output strides replaced (which=1).
static std::vector<Dim> packed(const std::vector<Dim> &V, int64_t per, int which)
{
    std::vector<Dim> r = V;
    int64_t s = per;
    for (int i = (int)r.size() - 1; i >= 0; --i) {
        if (which == 0) r[i].is = s;
        else r[i].os = s;
        s *= r[i].n;
    }
    return r;
}

static int64_t vprod(const std::vector<Dim> &V)
{
    int64_t t = 1;
    for (const Dim &d : V) t *= d.n;
    return t;
}

struct Split {
    int64_t m = 0, r = 0;
};

// Cooley-Tukey split n = m * r for a two-pass transform: both factors must be
// leaves whose column tiles fit the LDS budget; the most balanced split wins
// (the radix-sqrt(n) step of Section 3).
static bool choose_split(int64_t n, int prec, Split *sp)
{
    const int btmin = prec ? 4 : 8;
    int64_t best_m = 0;
    double best = 1e300;
    for (int64_t m = 2; m * m <= n * 64 && m < n; ++m) {
        if (n % m) continue;
        const int64_t r = n / m;
        if (!leaf_fits(m, prec, btmin) || !leaf_fits(r, prec, btmin)) continue;
        // most balanced split; of two mirror splits the one with the longer
        // first pass (a power-of-two first pass of 256 points or more runs in
        // the leaf kernel's transposing tiles)
        const double cost = std::fabs(std::log((double)m) - std::log((double)r));
        if (cost <= best) {
            best = cost;
            best_m = m;
        }
    }
    if (!best_m) return false;
    sp->m = best_m;
    sp->r = n / best_m;
    return true;
}

static int plan_line(Builder &b, Dim d, std::vector<Dim> V, int src, int dst, int64_t src_off,
                     int64_t dst_off, bool conj_in, bool conj_out);

// The plan's split of a length: a measured one when it is a valid split,
// else the estimate's.
static bool split_for(const PlanImpl *p, int64_t n, int prec, Split *sp)
{
    if (const StructChoice *c = choice_for(p, n)) {
        const int btmin = prec ? 4 : 8;
        const int64_t m = c->split;
        if (m > 1 && m < n && n % m == 0 && leaf_fits(m, prec, btmin) &&
            leaf_fits(n / m, prec, btmin)) {
            sp->m = m;
            sp->r = n / m;
            return true;
        }
    }
    return choose_split(n, prec, sp);
}

// ------------------------------------------------------------ convolution lengths
// Estimate-mode costs of the cyclic convolutions behind prime sizes: the
// relative cost per point of one stage of radix R inside a convolution (two
// transforms and the spectrum product in the generic tile kernel), fitted to
// convolutions of lengths 1050 to 131072 whose radices differ, measured on
// MI355X (FP32).  Powers of two cost about the same per stage; lengths with
// 11, 13 and 15 ran much slower per point.  The figures rank convolution
// lengths only: in plain transforms the same radices are not slow (3375 =
// 15^3 runs at the rate of a power of two, and choosing the radices of
// plain leaves by these figures made them slower).
static double stage_cost(int R)
{
    switch (R) {
    case 2: case 4: case 8: case 16: return 1.0;
    case 3: case 12: case 14: return 1.15;
    case 5: case 7: case 9: case 10: return 1.65;
    case 6: return 1.7;
    case 13: return 2.85;
    case 11: return 3.3;
    default: return 3.8;   // 15
    }
}

// A convolution split in three passes: each pass of the generic kernel
// costs kPassCost per point plus its stages (the outer passes one transform
// of the first factor, the middle pass two of the second); a pass that runs
// in the leaf kernel's column tiles (Bluestein only; outer factor a power of
// two in 256..2048, middle factor in 64..2048) costs kLeafPassCost.  Rader's
// index-table gather and scatter add kRaderTileCost per point inside a tile
// and kRaderSplitCost in the outer passes (random 8-byte accesses).  Fitted
// to three-pass convolutions of lengths 18432 to 131072 measured on MI355X.
constexpr double kPassCost = 1.3;
constexpr double kLeafPassCost = 1.26;
constexpr double kRaderTileCost = 1.0;
constexpr double kRaderSplitCost = 2.5;

static bool pow2_in(int64_t n, int64_t lo, int64_t hi)
{
    return (n & (n - 1)) == 0 && n >= lo && n <= hi;
}

// Estimated cost of a length-M convolution (forward transform, product,
// inverse transform), in units of one power-of-two stage of the generic
// kernel over M points; infinite when M has no plan.
static double conv_cost(int64_t M, int prec, bool rader)
{
    // Bluestein over a power-of-two length in one tile runs in the
    // specialized leaf kernel, whose stages cost about half as much
    // (measured: 12288 generic 0.70 ms, 16384 leaf 0.46 ms, 5582 x 6011)
    if (!rader && leaf_supported(prec, M)) {
        int st = 0;
        for (int64_t m = 1; m < M; m *= 16) ++st;
        return 0.5 * st * (double)M;
    }
    Leaf L;
    if (leaf_fits(M, prec, 1) && make_leaf_shape(M, 16, max_threads(prec), &L)) {
        double c = rader ? kRaderTileCost : 0.0;
        for (int R : L.rad) c += stage_cost(R);
        return c * (double)M;
    }
    Split sp;
    if (!choose_split(M, prec, &sp)) return HUGE_VAL;
    const int bt = prec ? 4 : 8;
    Leaf A, B;
    if (!make_leaf_shape(sp.m, 16, max_threads(prec) / bt, &A) ||
        !make_leaf_shape(sp.r, 16, max_threads(prec) / bt, &B))
        return HUGE_VAL;
    double sa = 0, sb = 0;
    for (int R : A.rad) sa += stage_cost(R);
    for (int R : B.rad) sb += stage_cost(R);
    const double outer = !rader && pow2_in(sp.m, 256, 2048) ? kLeafPassCost : kPassCost + 0.41 * sa;
    const double mid = !rader && pow2_in(sp.r, 64, 2048) ? kLeafPassCost : kPassCost + 0.81 * sb;
    return (2 * outer + mid + (rader ? kRaderSplitCost : 0.0)) * (double)M;
}

// Bluestein's convolution length: any M >= 2n-1 gives the same result.  The
// candidates are the smallest smooth M and the smallest of each form 2^a*k
// with odd k <= 15 (power-of-two stages and at most one other), up to the
// smallest power of two; the cheapest by conv_cost wins, ties to the shorter.
static int64_t bluestein_length(int64_t n, int prec, double *cost)
{
    const int64_t lo = 2 * n - 1;
    int64_t p2 = 1;
    while (p2 < lo) p2 <<= 1;
    std::vector<int64_t> cand;
    for (int64_t c = lo; c <= p2; ++c)
        if (is_smooth(c)) {
            cand.push_back(c);
            break;
        }
    for (int64_t k = 1; k <= 15; k += 2) {
        int64_t c = k;
        while (c < lo) c <<= 1;
        if (c <= p2 && is_smooth(c)) cand.push_back(c);
    }
    std::sort(cand.begin(), cand.end());
    int64_t best = 0;
    double bc = HUGE_VAL;
    for (int64_t c : cand) {
        const double k = conv_cost(c, prec, false);
        if (k < bc) {
            bc = k;
            best = c;
        }
    }
    *cost = bc;
    return best;
}

// Leaf: one pass.
static int plan_leaf(Builder &b, Dim d, const std::vector<Dim> &V, int src, int dst,
                     int64_t src_off, int64_t dst_off, bool conj_in, bool conj_out)
{
    LineSpec ls;
    ls.line = d;
    ls.V = V;
    ls.src = src;
    ls.dst = dst;
    ls.src_off = src_off;
    ls.dst_off = dst_off;
    ls.flags = (conj_in ? PF_CONJ_IN : 0) | (conj_out ? PF_CONJ_OUT : 0);
    ls.what = "leaf";
    return add_line_pass(b, ls);
}

// Cooley-Tukey DIT step, radix r = n/m (Section 4.2).
static int add_transpose_pass(Builder &b, int buf, int64_t off, int64_t q, int64_t rs, int64_t cs,
                              const std::vector<Dim> &V)
{
    Pass ps;
    ps.kind = 3;
    if (V.size() > 8) return fail(MFFT_ENOTSUP, "transpose over more than 8 loops");
    ps.t.elem_bytes = elem_bytes(b.p->prob.prec);
    ps.t.rank = (int)V.size();
    ps.t.q = q;
    ps.t.rs = rs;
    ps.t.cs = cs;
    ps.t.total = 1;
    for (size_t i = 0; i < V.size(); ++i) {
        ps.t.n[i] = V[i].n;
        ps.t.s[i] = V[i].is;
        ps.t.total *= V[i].n;
    }
    ps.src = ps.dst = buf;
    ps.src_off = ps.dst_off = off;
    ps.prec = b.p->prob.prec;
    ps.bytes = 2.0 * (double)(q * q) * ps.t.total * ps.t.elem_bytes;
    std::ostringstream d;
    d << "transpose q=" << q << " in place x" << ps.t.total;
    ps.desc = d.str();
    b.p->passes.push_back(ps);
    return MFFT_OK;
}

// In-place transpose of a rows x cols matrix of runs (run x = row*cols + col,
// `len` elements of stride s each, at x*len*s) into cols x rows: run x goes
// to (x mod cols)*rows + x div cols.  The cycles of the permutation are
// found on the host; a table of run destinations and one start per cycle go
// to the device.
static int add_run_transpose_pass(Builder &b, int buf, int64_t off, int64_t rows, int64_t cols,
                                  int64_t len, int64_t s, const std::vector<Dim> &V)
{
    PlanImpl *p = b.p;
    if (V.size() > 8) return fail(MFFT_ENOTSUP, "permutation over more than 8 loops");
    if (len > 2048) return fail(MFFT_ENOTSUP, "runs of more than 2048 elements");
    const int64_t items = rows * cols;
    if (items > INT32_MAX) return fail(MFFT_ENOTSUP, "too many runs");
    std::vector<int32_t> next(items), starts;
    for (int64_t x = 0; x < items; ++x) next[x] = (int32_t)((x % cols) * rows + x / cols);
    std::vector<char> seen(items, 0);
    for (int64_t x = 0; x < items; ++x) {
        if (seen[x]) continue;
        int64_t clen = 0;
        for (int64_t y = x; !seen[y]; y = next[y]) {
            seen[y] = 1;
            ++clen;
        }
        if (clen > 1) starts.push_back((int32_t)x);
    }
    if (starts.empty()) return MFFT_OK;   // identity (a single row or column of runs)
    int32_t *dnext = (int32_t *)table_alloc(p, (size_t)items * 4);
    int32_t *dstarts = (int32_t *)table_alloc(p, starts.size() * 4);
    if (!dnext || !dstarts) return fail(MFFT_ENOMEM, "permutation table allocation failed");
    hipError_t e = hipMemcpy(dnext, next.data(), (size_t)items * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dstarts, starts.data(), starts.size() * 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    Pass ps;
    ps.kind = 4;
    ps.pm.elem_bytes = elem_bytes(p->prob.prec);
    ps.pm.rank = (int)V.size();
    ps.pm.len = len;
    ps.pm.es = s;
    ps.pm.xs = len * s;
    ps.pm.next = dnext;
    ps.pm.starts = dstarts;
    ps.pm.ncycles = (int32_t)starts.size();
    ps.pm.nitems = (int32_t)items;
    ps.pm.total = 1;
    for (size_t i = 0; i < V.size(); ++i) {
        ps.pm.n[i] = V[i].n;
        ps.pm.s[i] = V[i].is;
        ps.pm.total *= V[i].n;
    }
    ps.src = ps.dst = buf;
    ps.src_off = ps.dst_off = off;
    ps.prec = p->prob.prec;
    ps.bytes = 2.0 * (double)(items * len) * ps.pm.total * ps.pm.elem_bytes;
    std::ostringstream d;
    d << "transpose " << rows << "x" << cols << " runs of " << len << " in place x" << ps.pm.total
      << " (" << starts.size() << " cycles)";
    ps.desc = d.str();
    p->passes.push_back(ps);
    return MFFT_OK;
}

// In-place Cooley-Tukey step without scratch (Section 4.2's in-place plans)
// for n = k*q*q, viewed as m = k*q rows of r = q columns: columns j
// (elements l*q + j, l < m) transformed in place with the twiddle
// w_n^(j*k1) on store, then rows k1 (elements k1*q + j) in place, which
// leaves Y[k1 + k2*m] at k1*q + k2 -- the m x q matrix whose transpose is the
// result.  It is transposed in place as k q x q blocks (each transposed in
// place) followed by a transpose of the k x q matrix of q-element runs
// (permutation cycles).  Every pass reads a tile's elements before writing
// them and tiles are disjoint, so no pass needs a copy of its input.
static int plan_ct_square_inplace(Builder &b, Dim d, const std::vector<Dim> &V, int buf,
                                  int64_t off, bool conj_in, bool conj_out)
{
    const int prec = b.p->prob.prec;
    const int64_t n = d.n;
    const int bt = prec ? 4 : 8;
    // the smallest k with n = k*q*q, q <= 2048 and both q and k*q one pass
    int64_t q = 0, m = 0, k = 0;
    for (int64_t f = 1; f <= 64 && !q; ++f) {
        if (n % f) continue;
        int64_t c = (int64_t)std::llround(std::sqrt((double)(n / f)));
        while (c > 0 && c * c > n / f) --c;
        while ((c + 1) * (c + 1) <= n / f) ++c;
        if (c > 1 && c * c == n / f && c <= 2048 && leaf_fits(c, prec, bt) &&
            leaf_fits(f * c, prec, bt)) {
            q = c;
            m = f * c;
            k = f;
        }
    }
    if (!q)
        return fail(MFFT_ENOTSUP,
                    "in place without scratch needs n = k*q*q with q and k*q one pass each");
    if (d.is != d.os) return fail(MFFT_ENOTSUP, "in place without scratch needs equal strides");
    for (const Dim &v : V)
        if (v.is != v.os) return fail(MFFT_ENOTSUP, "in place without scratch needs equal strides");
    const int64_t s = d.is, r = q;
    // columns j < r: elements l*r + j, l < m, in place, times w_n^(j*k1)
    LineSpec A;
    A.what = "ctA";
    A.line = {m, r * s, r * s};
    A.V = V;
    A.V.push_back({r, s, s});
    A.inner = (int)A.V.size() - 1;
    A.src = A.dst = buf;
    A.src_off = A.dst_off = off;
    A.flags = PF_TW4 | (conj_in ? PF_CONJ_IN : 0);
    A.tw4_N = n;
    int rc = add_line_pass(b, A);
    if (rc) return rc;
    // rows k1 < m: elements k1*r + j, in place; Y[k1 + m*k2] lands at k1*r + k2
    std::vector<Dim> VB = V;
    VB.push_back({m, r * s, r * s});
    rc = plan_line(b, Dim{r, s, s}, VB, buf, buf, off, off, false, conj_out);
    if (rc) return rc;
    if (k == 1) return add_transpose_pass(b, buf, off, q, q * s, s, V);
    // k blocks of q x q, each transposed in place: run i*q + c (c < q) then
    // holds the results Y[c*m + i*q ...] that belong at run c*k + i
    std::vector<Dim> VT = V;
    VT.push_back({k, q * q * s, q * q * s});
    rc = add_transpose_pass(b, buf, off, q, q * s, s, VT);
    if (rc) return rc;
    return add_run_transpose_pass(b, buf, off, k, q, q, s, V);
}

// In-place rank-0 transpose without scratch (Section 4.2, "Rank-0 plans":
// the in-place transpose as a rank-0 problem with two vector dimensions): an
// R x C matrix (rows of C elements of stride s) rewritten as its C x R
// transpose, with C = k*R or R = k*C: the k square blocks transposed in
// place, then a transpose of the matrix of runs (one shorter side each).
// Other vector loops (is = os) repeat it.
static int plan_rank0_transpose_inplace(Builder &b, const std::vector<Dim> &V)
{
    int ia = -1, ib = -1;
    for (size_t i = 0; i < V.size(); ++i)
        for (size_t j = 0; j < V.size(); ++j) {
            if (i == j) continue;
            const Dim &A = V[i], &B = V[j];   // A: rows (R), B: columns (C)
            const int64_t st = B.is;
            if (st > 0 && A.is == B.n * st && A.os == st && B.os == A.n * st) {
                ia = (int)i;
                ib = (int)j;
            }
        }
    if (ia < 0) return fail(MFFT_ENOTSUP, "in place without scratch: rank-0 problem is not a transpose");
    std::vector<Dim> outer;
    for (size_t i = 0; i < V.size(); ++i) {
        if ((int)i == ia || (int)i == ib) continue;
        if (V[i].is != V[i].os) return fail(MFFT_ENOTSUP, "in place without scratch: other loops move");
        outer.push_back(V[i]);
    }
    const int64_t R = V[ia].n, C = V[ib].n, st = V[ib].is;
    const int64_t q = std::min(R, C), k = std::max(R, C) / q;
    if (std::max(R, C) % q) return fail(MFFT_ENOTSUP, "in place without scratch: sides not multiples");
    if (q > 2048) return fail(MFFT_ENOTSUP, "in place without scratch: shorter side above 2048");
    std::vector<Dim> VT = outer;
    if (C >= R) {
        // blocks side by side: block i at columns i*q.. of every row
        if (k > 1) VT.push_back({k, q * st, q * st});
        int rc = add_transpose_pass(b, BUF_IN, 0, q, C * st, st, VT);
        if (rc || k == 1) return rc;
        // run a*k + i (row a, block i) holds output row i*q + a
        return add_run_transpose_pass(b, BUF_IN, 0, R, k, q, st, outer);
    }
    // blocks stacked: block i = rows i*q.. (contiguous)
    VT.push_back({k, q * C * st, q * C * st});
    int rc = add_transpose_pass(b, BUF_IN, 0, q, C * st, st, VT);
    if (rc) return rc;
    // run i*q + c (block i, row c) holds part i of output row c
    return add_run_transpose_pass(b, BUF_IN, 0, k, q, q, st, outer);
}

static int plan_ct(Builder &b, Dim d, const std::vector<Dim> &V, int src, int dst,
                   int64_t src_off, int64_t dst_off, bool conj_in, bool conj_out, Split sp)
{
    const int64_t n = d.n, m = sp.m, r = sp.r;
    const int eb = elem_bytes(b.p->prob.prec);
    const bool oop = !(src == dst && src_off == dst_off);
    LineSpec A;
    A.what = "ctA";
    A.flags = PF_TW4 | (conj_in ? PF_CONJ_IN : 0);
    A.tw4_N = n;
    A.src = src;
    A.src_off = src_off;
    if (oop && dst != BUF_IN) {
        // pass A straight into the output, pass B in place there
        A.line = {m, r * d.is, d.os};
        A.V = V;
        A.V.push_back({r, d.is, m * d.os});
        A.inner = (int)A.V.size() - 1;
        A.dst = dst;
        A.dst_off = dst_off;
        int rc = add_line_pass(b, A);
        if (rc) return rc;
        Dim dB{r, m * d.os, m * d.os};
        std::vector<Dim> VB = copy_o(V);
        VB.push_back({m, d.os, d.os});
        return plan_line(b, dB, VB, dst, dst, dst_off, dst_off, false, conj_out);
    }
    if (b.p->flags & MFFT_NO_SCRATCH) {
        if (oop) return fail(MFFT_ENOTSUP, "no plan without scratch memory for this problem");
        return plan_ct_square_inplace(b, d, V, src, src_off, conj_in, conj_out);
    }
    // in place: pass A into packed scratch (transform v at v*n, element l2*m + k1)
    const int64_t H = vprod(V);
    const int64_t off = b.scratch_take(H * n * eb) / eb;
    A.line = {m, r * d.is, 1};
    A.V = packed(V, n, 1);
    A.V.push_back({r, d.is, m});
    A.inner = (int)A.V.size() - 1;
    A.dst = BUF_SCRATCH;
    A.dst_off = off;
    int rc = add_line_pass(b, A);
    if (rc) return rc;
    Dim dB{r, m, m * d.os};
    std::vector<Dim> VB = packed(V, n, 0);
    VB.push_back({m, 1, d.os});
    return plan_line(b, dB, VB, BUF_SCRATCH, dst, off, dst_off, false, conj_out);
}

// Rader's algorithm for prime p (Section 4.2, "Plans for prime sizes"):
// Y[0] = sum x; Y[g^-q] = x0 + sum_j x[g^j] w_p^(g^(j-q)), a cyclic
// convolution of length p-1 evaluated by FFT, pointwise product with the
// precomputed DFT of b_m = w_p^(g^-m), and inverse FFT.
static int rader_tables(Builder &b, int64_t pr, int32_t **gather, int32_t **scatter,
                        void **spec);
static int bluestein_tables(Builder &b, int64_t n, int64_t M, void **chirp, void **spec);

// The middle pass of a three-pass convolution reads spectrum entry k1 + k2*m1
// for element k2 of line k1; consecutive lanes work on consecutive k2, so the
// pass reads a copy stored line by line (k1*r1 + k2), one coalesced run per
// line instead of one cache line per element.
static int spectrum_by_line(Builder &b, const void *spec, int64_t m1, int64_t r1, void **out)
{
    PlanImpl *p = b.p;
    const int eb = elem_bytes(p->prob.prec);
    *out = table_alloc(p, (size_t)(m1 * r1) * eb);
    if (!*out) return fail(MFFT_ENOMEM, "spectrum table allocation failed");
    CopyArgs c{};
    c.in = spec;
    c.out = *out;
    c.rank = 2;
    c.elem_bytes = eb;
    c.total = m1 * r1;
    c.n[0] = m1;   // k1
    c.is[0] = 1;
    c.os[0] = r1;
    c.n[1] = r1;   // k2
    c.is[1] = m1;
    c.os[1] = 1;
    hipError_t e = launch_copy(c, p->stream);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    return MFFT_OK;
}

static int plan_rader(Builder &b, Dim d, const std::vector<Dim> &V, int src, int dst,
                      int64_t src_off, int64_t dst_off, bool conj_in, bool conj_out)
{
    const int64_t pr = d.n, L = pr - 1;
    const int eb = elem_bytes(b.p->prob.prec);
    int32_t *gat, *sct;
    void *spec;
    int rc = rader_tables(b, pr, &gat, &sct, &spec);
    if (rc) return rc;
    const int btmin = b.p->prob.prec ? 4 : 8;
    if (leaf_fits(L, b.p->prob.prec, 1)) {
        LineSpec ls;
        ls.what = "rader";
        ls.line = d;
        ls.conv_n = L;
        ls.V = V;
        ls.src = src;
        ls.dst = dst;
        ls.src_off = src_off;
        ls.dst_off = dst_off;
        ls.flags = PF_CONV | PF_RADER | PF_GATHER | PF_SCATTER | PF_CONJ_A |
                   (conj_in ? PF_CONJ_IN : 0) | (conj_out ? PF_CONJ_OUT : 0);
        ls.li_lim = L;
        ls.lo_lim = L;
        ls.gather = gat;
        ls.scatter = sct;
        ls.conv = spec;
        if (src == dst && src_off == dst_off && d.is != d.os)
            return fail(MFFT_ENOTSUP, "in-place Rader needs equal strides");
        return add_line_pass(b, ls);
    }
    Split sp;
    if (!split_for(b.p, L, b.p->prob.prec, &sp)) return fail(MFFT_ENOTSUP, "Rader length too large");
    (void)btmin;
    const int64_t m1 = sp.m, r1 = sp.r;
    const int64_t H = vprod(V);
    const int64_t s0 = b.scratch_take(H * L * eb) / eb;
    const int64_t s1 = b.scratch_take(H * L * eb) / eb;
    const int64_t aux = b.scratch_take(H * 2 * eb);
    std::vector<Dim> Vp = packed(V, L, 1);   // outputs packed in scratch
    // P1: DIT pass A over a[li] = x[g^li], li = c + l*r1 (c < r1), twiddled; saves x0
    LineSpec A;
    A.what = "raderA";
    A.line = {m1, d.is, 1};
    A.V = V;
    for (size_t i = 0; i < A.V.size(); ++i) A.V[i].os = Vp[i].os;
    A.V.push_back({r1, 0, m1});
    A.inner = (int)A.V.size() - 1;
    A.src = src;
    A.src_off = src_off;
    A.dst = BUF_SCRATCH;
    A.dst_off = s0;
    A.flags = PF_GATHER | PF_TW4 | PF_AUX_X0 | PF_XCD | (conj_in ? PF_CONJ_IN : 0);
    A.gather = gat;
    A.li_c = 1;
    A.li_l = r1;
    A.li_lim = L;
    A.tw4_N = L;
    A.aux_off = aux;
    rc = add_line_pass(b, A);
    if (rc) return rc;
    // P2: on the same lines k1 (stride m1): the forward r1-point DFTs (DIT pass B),
    // the pointwise product with the spectrum (index k1 + k2*m1), and the first
    // step of the inverse transform in decimation-in-frequency order (r1-point
    // DFTs of the conjugate, then the twiddle w_L^(k1*j1)); saves the zero
    // frequency of line 0.  Stored at j1*m1 + k1.
    LineSpec B;
    B.what = "raderB";
    B.line = {r1, m1, m1};
    B.V = packed(packed(V, L, 0), L, 1);
    B.V.push_back({m1, 1, 1});
    B.inner = (int)B.V.size() - 1;
    B.src = BUF_SCRATCH;
    B.src_off = s0;
    B.dst = BUF_SCRATCH;
    B.dst_off = s1;
    B.flags = PF_CONV | PF_TW4 | PF_AUX_A0;
    void *spec_lines = nullptr;
    rc = spectrum_by_line(b, spec, m1, r1, &spec_lines);
    if (rc) return rc;
    B.conv = spec_lines;
    B.conv_c = r1;
    B.conv_k = 1;
    B.tw4_N = L;
    B.aux_off = aux;
    rc = add_line_pass(b, B);
    if (rc) return rc;
    // P3: inverse, second step: m1-point DFTs over k1 (contiguous rows j1), back
    // from the conjugate, add x0, scatter Y[g^-q] for q = j1 + j2*r1; Y[0] = x0 + A0
    LineSpec D;
    D.what = "raderC";
    D.line = {m1, 1, d.os};
    D.V = packed(V, L, 0);
    D.V.push_back({r1, m1, 0});
    D.inner = (int)D.V.size() - 1;
    D.src = BUF_SCRATCH;
    D.src_off = s1;
    D.dst = dst;
    D.dst_off = dst_off;
    D.flags = PF_CONJ_A | PF_AUX_ADD | PF_SCATTER | PF_XCD | PF_NT_IN |
              (conj_out ? PF_CONJ_OUT : 0);
    D.scatter = sct;
    D.lo_c = 1;
    D.lo_k = r1;
    D.lo_lim = L;
    D.aux_off = aux;
    return add_line_pass(b, D);
}

// Bluestein: Y_k = c_k sum_l (x_l c_l) conj(c_(k-l)), c_k = w_(2n)^(k^2 mod 2n),
// a linear convolution done as a cyclic one of length M >= 2n-1.
static int plan_bluestein(Builder &b, Dim d, const std::vector<Dim> &V, int src, int dst,
                          int64_t src_off, int64_t dst_off, bool conj_in, bool conj_out)
{
    const int64_t n = d.n;
    const int prec = b.p->prob.prec;
    const int eb = elem_bytes(prec);
    double cost;
    int64_t M = bluestein_length(n, prec, &cost);
    if (const StructChoice *c = choice_for(b.p, n)) {
        // a measured convolution length: any smooth M >= 2n-1 with a plan
        Split t;
        if (c->M >= 2 * n - 1 && is_smooth(c->M) &&
            (leaf_fits(c->M, prec, 1) || choose_split(c->M, prec, &t))) {
            M = c->M;
            cost = 0;
        }
    }
    if (!M || cost == HUGE_VAL) return fail(MFFT_ENOTSUP, "no Bluestein length");
    const bool single = leaf_fits(M, prec, 1);
    void *chirp, *spec;
    int rc = bluestein_tables(b, n, M, &chirp, &spec);
    if (rc) return rc;
    if (single) {
        LineSpec ls;
        ls.what = "bluestein";
        ls.line = d;
        ls.conv_n = M;
        ls.V = V;
        ls.src = src;
        ls.dst = dst;
        ls.src_off = src_off;
        ls.dst_off = dst_off;
        ls.flags = PF_CONV | PF_PRE_MUL | PF_POST_MUL | PF_CONJ_A | (conj_in ? PF_CONJ_IN : 0) |
                   (conj_out ? PF_CONJ_OUT : 0);
        ls.li_lim = n;
        ls.lo_lim = n;
        ls.pre = chirp;
        ls.post = chirp;
        ls.conv = spec;
        if (src == dst && src_off == dst_off && d.is != d.os)
            return fail(MFFT_ENOTSUP, "in-place Bluestein needs equal strides");
        return add_line_pass(b, ls);
    }
    Split sp;
    if (!split_for(b.p, M, prec, &sp)) return fail(MFFT_ENOTSUP, "no split of the Bluestein length");
    const int64_t m1 = sp.m, r1 = sp.r;
    const int64_t H = vprod(V);
    const int64_t s0 = b.scratch_take(H * M * eb) / eb;
    const int64_t s1 = b.scratch_take(H * M * eb) / eb;
    std::vector<Dim> Vp = packed(V, M, 1);
    // P1: chirp multiply, zero padding, DIT pass A of the length-M transform
    LineSpec A;
    A.what = "bluesteinA";
    A.line = {m1, r1 * d.is, 1};
    A.V = V;
    for (size_t i = 0; i < A.V.size(); ++i) A.V[i].os = Vp[i].os;
    A.V.push_back({r1, d.is, m1});
    A.inner = (int)A.V.size() - 1;
    A.src = src;
    A.src_off = src_off;
    A.dst = BUF_SCRATCH;
    A.dst_off = s0;
    A.flags = PF_PRE_MUL | PF_TW4 | (conj_in ? PF_CONJ_IN : 0);
    A.pre = chirp;
    A.li_c = 1;
    A.li_l = r1;
    A.li_lim = n;
    A.tw4_N = M;
    rc = add_line_pass(b, A);
    if (rc) return rc;
    // P2: DIT pass B, spectrum product (index k1 + k2*m1), first
    // decimation-in-frequency step of the inverse, twiddle; stored at j1*m1 + k1
    LineSpec B;
    B.what = "bluesteinB";
    B.line = {r1, m1, m1};
    B.V = packed(packed(V, M, 0), M, 1);
    B.V.push_back({m1, 1, 1});
    B.inner = (int)B.V.size() - 1;
    B.src = BUF_SCRATCH;
    B.src_off = s0;
    B.dst = BUF_SCRATCH;
    B.dst_off = s1;
    B.flags = PF_CONV | PF_TW4;
    void *spec_lines = nullptr;
    rc = spectrum_by_line(b, spec, m1, r1, &spec_lines);
    if (rc) return rc;
    B.conv = spec_lines;
    B.conv_c = r1;
    B.conv_k = 1;
    B.conv_cols = spec;   // entry k1 + k2*m1: line k1, element k2
    B.conv_cols_c = 1;
    B.conv_cols_k = m1;
    B.tw4_N = M;
    rc = add_line_pass(b, B);
    if (rc) return rc;
    // P3: second inverse step over contiguous rows, back from the conjugate,
    // chirp multiply, keep outputs j = j1 + j2*r1 < n
    LineSpec D;
    D.what = "bluesteinC";
    D.line = {m1, 1, r1 * d.os};
    D.V = packed(V, M, 0);
    D.V.push_back({r1, m1, d.os});
    D.inner = (int)D.V.size() - 1;
    D.src = BUF_SCRATCH;
    D.src_off = s1;
    D.dst = dst;
    D.dst_off = dst_off;
    D.flags = PF_CONJ_A | PF_POST_MUL | (conj_out ? PF_CONJ_OUT : 0);
    D.post = chirp;
    D.lo_c = 1;
    D.lo_k = r1;
    D.lo_lim = n;
    return add_line_pass(b, D);
}

static int plan_line(Builder &b, Dim d, std::vector<Dim> V, int src, int dst, int64_t src_off,
                     int64_t dst_off, bool conj_in, bool conj_out)
{
    const int prec = b.p->prob.prec;
    const int64_t n = d.n;
    // lengths with radices 17, 19, 23 take the plain Cooley-Tukey path too when
    // they fit a leaf or split into two leaves (else the paths for large
    // prime factors below)
    Split wsp;
    const bool wide_ok = !is_smooth(n) && is_smooth23(n) &&
                         (leaf_fits(n, prec, 1) || split_for(b.p, n, prec, &wsp));
    if (is_smooth(n) || wide_ok) {
        const bool strided = std::llabs(d.is) != 1 || std::llabs(d.os) != 1;
        if (leaf_fits(n, prec, strided ? (prec ? 4 : 8) : 1) || leaf_fits(n, prec, 1) ||
            (!strided && wide_leaf_fits(n, prec) && !(choice_for(b.p, n) && choice_for(b.p, n)->split))) {
            const bool inplace = src == dst && src_off == dst_off;
            if (!inplace || d.is == d.os)
                return plan_leaf(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out);
        }
        Split sp;
        if (!split_for(b.p, n, prec, &sp)) {
            // three or more passes: peel the largest leaf factor and recurse
            int64_t best = 0;
            for (int64_t m = 2; m < n; ++m)
                if (n % m == 0 && leaf_fits(m, prec, prec ? 4 : 8)) best = m;
            if (!best) return fail(MFFT_ENOTSUP, "no Cooley-Tukey split");
            sp.m = best;
            sp.r = n / best;
        }
        return plan_ct(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out, sp);
    }
    // Rader's convolution has the fixed length p-1; above 256 points
    // Bluestein's, at least twice as long, wins when it runs in the leaf
    // kernel or p-1 needs costly radices (both estimated by conv_cost;
    // measured: 1009 Rader 0.45 ms, Bluestein 0.27 ms, 33254 transforms;
    // 97 Rader 0.27 ms, Bluestein 0.31 ms)
    if (smallest_prime_factor(n) == n && is_smooth(n - 1)) {
        const StructChoice *c = choice_for(b.p, n);
        if (c && c->prime == 1) return plan_rader(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out);
        double blue = HUGE_VAL;
        if (n > 256) (void)bluestein_length(n, prec, &blue);
        if ((!c || c->prime != 2) && (n <= 256 || conv_cost(n - 1, prec, true) <= blue))
            return plan_rader(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out);
        if (c && c->prime == 2)
            return plan_bluestein(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out);
    }
    // A composite length whose only prime factor above 13 is p, once: one
    // Cooley-Tukey step (eq. ct) with smooth m-point transforms first (m the
    // largest divisor of n/p that a column pass takes) and r = n/m-point DFTs
    // second, r a multiple of p planned in one tile (Rader or Bluestein),
    // instead of Bluestein over the whole length -- two passes over n rather
    // than three over a convolution of at least 2n.  Taken when that
    // convolution would not fit one tile (Bluestein in one kernel is one pass)
    // and r <= 2048.  Measured (FP32/FP64, 256 MiB batches): 17*4096 1.53 ->
    // 0.84 ms, 31*1024 0.93 -> 0.42, 17*1024 FP64 1.95 -> 0.63; but 4099*8,
    // whose second pass is a 4099-point Bluestein in one tile, 1.47 -> 1.87.
    if (smallest_prime_factor(n) != n) {
        int64_t q = n, pmax = 1;
        for (int64_t f = 2; f * f <= q; ++f)
            while (q % f == 0) {
                pmax = f;
                q /= f;
            }
        if (q > 1) pmax = q;
        const int64_t s = n / pmax;
        int64_t m = 0;
        if (is_smooth(s))
            for (int64_t c = std::min<int64_t>(s, 16384); c >= 2 && !m; --c)
                if (s % c == 0 && leaf_fits(c, prec, prec ? 4 : 8)) m = c;
        double c;
        const int64_t r = m ? n / m : 0;
        const bool whole_single = leaf_fits(bluestein_length(n, prec, &c), prec, 1);
        const bool r_single =
            m && ((r == pmax && is_smooth(r - 1) && leaf_fits(r - 1, prec, 1)) ||
                  leaf_fits(bluestein_length(r, prec, &c), prec, 1));
        if (!whole_single && r_single && r <= 2048) {
            Split sp;
            sp.m = m;
            sp.r = r;
            return plan_ct(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out, sp);
        }
    }
    return plan_bluestein(b, d, V, src, dst, src_off, dst_off, conj_in, conj_out);
}

// ------------------------------------------------------------ tables for primes

static int rader_tables(Builder &b, int64_t pr, int32_t **gather, int32_t **scatter, void **spec)
{
    PlanImpl *p = b.p;
    const int64_t L = pr - 1;
    const int64_t g = primitive_root(pr);
    if (!g) return fail(MFFT_ENOTSUP, "no primitive root");
    *gather = (int32_t *)table_alloc(p, (size_t)L * 4);
    *scatter = (int32_t *)table_alloc(p, (size_t)L * 4);
    *spec = table_alloc(p, (size_t)L * elem_bytes(p->prob.prec));
    void *bseq = dev_alloc(p, (size_t)L * 16);
    void *bhat = dev_alloc(p, (size_t)L * 16);
    if (!*gather || !*scatter || !*spec || !bseq || !bhat)
        return fail(MFFT_ENOMEM, "Rader table allocation failed");
    hipError_t e = launch_gen_rader(*gather, *scatter, bseq, pr, g, p->stream);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    // DFT of b in FP64 with this library, then scale by 1/(p-1) and round
    mfft_plan sub = nullptr;
    mfft_iodim dim{L, 1, 1};
    // the sub-plan takes its memory where this plan does (a caller's
    // allocator: no hipMalloc / hipFree, which can stall other threads'
    // launches, while a server plans beside its running requests)
    int rc = plan_internal(&sub, 1, &dim, 0, nullptr, 0, -1, MFFT_C64, p->stream, 0,
                           p->has_alloc ? &p->alloc : nullptr);
    if (rc) return rc;
    rc = mfft_execute(sub, bseq, bhat, (void *)p->stream);
    if (rc) {
        mfft_plan_destroy(sub);
        return rc;
    }
    e = launch_convert_scale(*spec, p->prob.prec, bhat, L, 1.0 / (double)L, p->stream);
    (void)hipStreamSynchronize(p->stream);
    mfft_plan_destroy(sub);
    dev_free(p, bseq, (size_t)L * 16);
    dev_free(p, bhat, (size_t)L * 16);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    return MFFT_OK;
}

static int bluestein_tables(Builder &b, int64_t n, int64_t M, void **chirp, void **spec)
{
    PlanImpl *p = b.p;
    const int prec = p->prob.prec;
    *chirp = table_alloc(p, (size_t)n * elem_bytes(prec));
    *spec = table_alloc(p, (size_t)M * elem_bytes(prec));
    void *c64 = dev_alloc(p, (size_t)n * 16);
    void *v = dev_alloc(p, (size_t)M * 16);
    void *vhat = dev_alloc(p, (size_t)M * 16);
    if (!*chirp || !*spec || !c64 || !v || !vhat)
        return fail(MFFT_ENOMEM, "Bluestein table allocation failed");
    hipError_t e = launch_gen_chirp(c64, n, p->stream);
    if (e == hipSuccess) e = launch_gen_bluestein_v(v, c64, n, M, p->stream);
    if (e == hipSuccess) e = launch_convert_scale(*chirp, prec, c64, n, 1.0, p->stream);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    mfft_plan sub = nullptr;
    mfft_iodim dim{M, 1, 1};
    // the sub-plan takes its memory where this plan does (a caller's
    // allocator: no hipMalloc / hipFree, which can stall other threads'
    // launches, while a server plans beside its running requests)
    int rc = plan_internal(&sub, 1, &dim, 0, nullptr, 0, -1, MFFT_C64, p->stream, 0,
                           p->has_alloc ? &p->alloc : nullptr);
    if (rc) return rc;
    rc = mfft_execute(sub, v, vhat, (void *)p->stream);
    if (rc) {
        mfft_plan_destroy(sub);
        return rc;
    }
    e = launch_convert_scale(*spec, prec, vhat, M, 1.0 / (double)M, p->stream);
    (void)hipStreamSynchronize(p->stream);
    mfft_plan_destroy(sub);
    dev_free(p, c64, (size_t)n * 16);
    dev_free(p, v, (size_t)M * 16);
    dev_free(p, vhat, (size_t)M * 16);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    return MFFT_OK;
}

// ------------------------------------------------------------ structural candidates
// (measure mode: Section 4.3's planner times alternatives instead of trusting
// the estimate)

// Radix sequences of a one-pass leaf of length n: the multisets of compiled
// radices with product n whose stages each fit the thread budget, with at most
// one stage more than the fewest, ordered by stages then thread need; each
// with its radices largest first, the estimate's sequence first of all, and the
// smallest-first order of the two best.
static std::vector<std::vector<int>> radix_candidates(int64_t n, int prec, size_t limit)
{
    static const int kRad[] = {23, 19, 17, 16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2};
    const int emax = leaf_emax(n);
    const int mt = max_threads(prec, emax);
    std::vector<std::vector<int>> all;
    std::vector<int> cur;
    std::function<void(int64_t, int)> rec = [&](int64_t rest, int from) {
        if (all.size() > 400 || (int)cur.size() > kMaxStages) return;
        if (rest == 1) {
            if (!cur.empty()) all.push_back(cur);
            return;
        }
        for (int i = from; i < 18; ++i) {
            const int R = kRad[i];
            if (rest % R || stage_threads(n, R, emax) > mt) continue;
            cur.push_back(R);
            rec(rest / R, i);
            cur.pop_back();
        }
    };
    rec(n, 0);
    if (all.empty()) return {};
    size_t fewest = SIZE_MAX;
    for (auto &r : all) fewest = std::min(fewest, r.size());
    auto need = [&](const std::vector<int> &r) {
        int t = 0;
        for (int R : r) t = std::max(t, stage_threads(n, R, emax));
        return t;
    };
    std::vector<std::vector<int>> keep;
    for (auto &r : all)
        if (r.size() <= fewest + 1) keep.push_back(r);
    std::stable_sort(keep.begin(), keep.end(), [&](const std::vector<int> &a, const std::vector<int> &b) {
        if (a.size() != b.size()) return a.size() < b.size();
        return need(a) < need(b);
    });
    std::vector<std::vector<int>> out;
    std::vector<int> est;
    if (radices_for(n, emax, mt, &est)) out.push_back(est);
    for (auto &r : keep) {
        if (out.size() >= limit) break;
        if (std::find(out.begin(), out.end(), r) == out.end()) out.push_back(r);
    }
    const size_t base = out.size();
    for (size_t i = 0; i < std::min<size_t>(2, base) && out.size() < limit + 2; ++i) {
        std::vector<int> up(out[i].rbegin(), out[i].rend());
        if (std::find(out.begin(), out.end(), up) == out.end()) out.push_back(up);
    }
    return out;
}

// The estimate's structural choice for lines of length n, spelled out (so
// that stored wisdom keeps it even if the estimate changes).
static StructChoice estimate_choice(const PlanImpl *p, int64_t n)
{
    const int prec = p->prob.prec;
    StructChoice c;
    if (n < 2) return c;
    if (smallest_prime_factor(n) == n) {
        if (n <= 23) return c;   // a radix: one butterfly
        double blue = HUGE_VAL;
        const int64_t M = bluestein_length(n, prec, &blue);
        if (is_smooth(n - 1) && (n <= 256 || conv_cost(n - 1, prec, true) <= blue)) {
            c.prime = 1;
        } else if (M) {
            c.prime = 2;
            c.M = M;
        }
        return c;
    }
    if (!is_smooth23(n)) return c;
    if (leaf_fits(n, prec, 1) || wide_leaf_fits(n, prec)) {
        if (leaf_supported(prec, n)) return c;
        // (a unit-stride line of a batch: the estimate's elements per thread)
        const int emax = wide_range(n) && prefer_wide(n, prec, 0) ? 24 : leaf_emax(n);
        Leaf L;
        if (make_leaf_shape(n, emax, max_threads(prec, emax), &L)) {
            c.rad = L.rad;
            c.bt = row_lines_per_tile(L.n, L.tpt, prec, 0, emax);
            if (wide_range(n)) c.emax = emax;
        }
        return c;
    }
    Split sp;
    if (choose_split(n, prec, &sp)) c.split = sp.m;
    return c;
}

std::vector<StructChoice> structure_candidates(const PlanImpl *p, int64_t n)
{
    const int prec = p->prob.prec;
    std::vector<StructChoice> out;
    out.push_back(estimate_choice(p, n));   // the estimate's, first
    if (n < 2) return out;
    if (smallest_prime_factor(n) == n) {
        if (n <= 23) return out;   // a radix: one butterfly
        if (is_smooth(n - 1)) {
            StructChoice c;
            c.prime = 1;
            out.push_back(c);
        }
        // Bluestein over each convolution length the estimate considers
        const int64_t lo = 2 * n - 1;
        int64_t p2 = 1;
        while (p2 < lo) p2 <<= 1;
        std::vector<int64_t> cand;
        for (int64_t c = lo; c <= p2; ++c)
            if (is_smooth(c)) {
                cand.push_back(c);
                break;
            }
        for (int64_t k = 1; k <= 15; k += 2) {
            int64_t c = k;
            while (c < lo) c <<= 1;
            if (c <= p2 && is_smooth(c) && std::find(cand.begin(), cand.end(), c) == cand.end())
                cand.push_back(c);
        }
        for (int64_t M : cand) {
            Split t;
            if (!leaf_fits(M, prec, 1) && !choose_split(M, prec, &t)) continue;
            StructChoice c;
            c.prime = 2;
            c.M = M;
            out.push_back(c);
        }
        return out;
    }
    if (!is_smooth23(n)) return out;
    if (wide_leaf_fits(n, prec)) {
        // one pass with 24 or 16 elements per thread (radices and lines per
        // tile as the estimate shapes them), and the two-pass splits below
        for (int e : {24, 16}) {
            Leaf L;
            if (!make_leaf_shape(n, e, max_threads(prec, e), &L)) continue;
            StructChoice c;
            c.emax = e;
            out.push_back(c);
        }
    }
    if (leaf_fits(n, prec, 1)) {
        // one pass; powers of two run in the specialized leaf kernel (fixed
        // radices), the rest in the generic kernel
        if (leaf_supported(prec, n)) return out;
        const auto rads = radix_candidates(n, prec, 6);
        for (size_t i = 0; i < rads.size(); ++i) {
            StructChoice c;
            c.rad = rads[i];
            if (i > 0) {
                out.push_back(c);
                continue;
            }
            // the estimate's radices (first) with other line counts per tile
            Leaf L;
            const int mt = max_threads(prec, leaf_emax(n));
            if (!leaf_shape_from(n, leaf_emax(n), mt, c.rad, &L)) continue;
            const int bt = row_lines_per_tile(L.n, L.tpt, prec, 0);
            for (int b2 : {bt / 2, bt * 2}) {
                if (b2 < 1 || b2 == bt || b2 * L.tpt > mt ||
                    tile_lds_bytes(L.n, b2, prec, L.emax) > g_lds_budget)
                    continue;
                StructChoice cb = c;
                cb.bt = b2;
                out.push_back(cb);
            }
        }
        return out;
    }
    // two passes: the splits whose factors are both column leaves, most
    // balanced first
    const int btmin = prec ? 4 : 8;
    std::vector<std::pair<double, int64_t>> sp;
    for (int64_t m = 2; m < n; ++m) {
        if (n % m || !leaf_fits(m, prec, btmin) || !leaf_fits(n / m, prec, btmin)) continue;
        sp.push_back({std::fabs(std::log((double)m) - std::log((double)(n / m))), m});
    }
    std::sort(sp.begin(), sp.end());
    for (size_t i = 0; i < sp.size() && i < 6; ++i) {
        StructChoice c;
        c.split = sp[i].second;
        out.push_back(c);
    }
    return out;
}

// "n=<length>[:r=<R>.<R>...][:b=<lines>][:s=<split>][:a=R|B][:M=<length>][:e=16|24]"
std::string choice_text(int64_t n, const StructChoice &c)
{
    std::ostringstream s;
    s << "n=" << n;
    if (!c.rad.empty()) {
        s << ":r=";
        for (size_t i = 0; i < c.rad.size(); ++i) s << (i ? "." : "") << c.rad[i];
    }
    if (c.bt) s << ":b=" << c.bt;
    if (c.split) s << ":s=" << c.split;
    if (c.prime) s << ":a=" << (c.prime == 1 ? "R" : "B");
    if (c.M) s << ":M=" << c.M;
    if (c.emax) s << ":e=" << c.emax;
    return s.str();
}

bool parse_choice(const std::string &text, int64_t *n, StructChoice *c)
{
    *c = StructChoice{};
    std::istringstream s(text);
    std::string f;
    bool have_n = false;
    while (std::getline(s, f, ':')) {
        if (f.size() < 3 || f[1] != '=') return false;
        const std::string v = f.substr(2);
        char *end = nullptr;
        switch (f[0]) {
        case 'n':
            *n = std::strtoll(v.c_str(), &end, 10);
            have_n = *end == 0 && *n > 1;
            break;
        case 'r': {
            std::istringstream rs(v);
            std::string r;
            while (std::getline(rs, r, '.')) {
                char *rend = nullptr;
                const long R = std::strtol(r.c_str(), &rend, 10);
                if (*rend || R < 2 || R > 23) return false;
                c->rad.push_back((int)R);
            }
            break;
        }
        case 'b': c->bt = (int)std::strtol(v.c_str(), &end, 10); break;
        case 's': c->split = std::strtoll(v.c_str(), &end, 10); break;
        case 'a':
            if (v == "R") c->prime = 1;
            else if (v == "B") c->prime = 2;
            else return false;
            break;
        case 'M': c->M = std::strtoll(v.c_str(), &end, 10); break;
        case 'e':
            c->emax = (int)std::strtol(v.c_str(), &end, 10);
            if (c->emax != 16 && c->emax != 24) return false;
            break;
        default: return false;
        }
        if (end && *end) return false;
    }
    return have_n && c->bt >= 0 && c->split >= 0 && c->M >= 0;
}

// The structural part of a choice string ("-" or "n=...;n=...").
bool parse_structure(const std::string &text, std::map<int64_t, StructChoice> *out)
{
    out->clear();
    if (text == "-" || text.empty()) return true;
    std::istringstream s(text);
    std::string item;
    while (std::getline(s, item, ';')) {
        int64_t n = 0;
        StructChoice c;
        if (!parse_choice(item, &n, &c)) return false;
        (*out)[n] = c;
    }
    return true;
}

// ------------------------------------------------------------ whole problems

static int add_copy_pass(Builder &b, const std::vector<Dim> &dims, int src, int dst,
                         int64_t src_off, int64_t dst_off, const char *what)
{
    Pass ps;
    ps.kind = 1;
    if (dims.size() > 8) return fail(MFFT_ENOTSUP, "copy of rank > 8");
    ps.c.rank = (int)dims.size();
    ps.c.elem_bytes = elem_bytes(b.p->prob.prec);
    ps.c.total = 1;
    for (size_t i = 0; i < dims.size(); ++i) {
        ps.c.n[i] = dims[i].n;
        ps.c.is[i] = dims[i].is;
        ps.c.os[i] = dims[i].os;
        ps.c.total *= dims[i].n;
    }
    ps.src = src;
    ps.dst = dst;
    ps.src_off = src_off;
    ps.dst_off = dst_off;
    ps.bytes = 2.0 * (double)ps.c.total * ps.c.elem_bytes;
    std::ostringstream d;
    d << what << " elements=" << ps.c.total;
    ps.desc = d.str();
    b.p->passes.push_back(ps);
    return MFFT_OK;
}

// ------------------------------------------------------------ real data

static int add_real_pass(Builder &b, int mode, int64_t n, int64_t cnt, int64_t is, int64_t os,
                         const std::vector<Dim> &V, int src, int64_t src_off, int dst,
                         int64_t dst_off, const void *tw, const char *what)
{
    Pass ps;
    ps.kind = 2;
    ps.prec = b.p->prob.prec;
    if (V.size() > 8) return fail(MFFT_ENOTSUP, "more than 8 vector loops");
    RealArgs &r = ps.r;
    r.mode = mode;
    r.n = n;
    r.cnt = cnt;
    r.is = is;
    r.os = os;
    r.tw = tw;
    r.vrank = (int)V.size();
    int64_t lines = 1;
    for (size_t i = 0; i < V.size(); ++i) {
        r.vn[i] = V[i].n;
        r.vis[i] = V[i].is;
        r.vos[i] = V[i].os;
        lines *= V[i].n;
    }
    r.total = lines * cnt;
    ps.src = src;
    ps.dst = dst;
    ps.src_off = src_off;
    ps.dst_off = dst_off;
    const double eb = elem_bytes(ps.prec);
    const double per_line = mode == RK_UNTANGLE ? (n / 2) * eb + (n / 2 + 1) * eb
                            : mode == RK_TANGLE ? (n / 2 + 1) * eb + (n / 2) * eb
                            : mode == RK_WIDEN  ? n * eb / 2 + n * eb
                            : mode == RK_HERM   ? (n / 2 + 1) * eb + n * eb
                                                : n * eb + n * eb / 2;
    ps.bytes = per_line * (double)lines;
    std::ostringstream d;
    d << what << " n=" << n << " lines=" << lines;
    ps.desc = d.str();
    b.p->passes.push_back(ps);
    return MFFT_OK;
}

// Real-data plans.  Even n with unit stride on the real side: the real
// sequence is read as n/2 complex values x[2j] + i x[2j+1] (no copy), so the
// transform costs a complex DFT of half the length plus one elementwise pass
// that separates (or, inverse, combines) the even and odd halves (a radix-2
// DIT step of eq. ct).  Otherwise the real data is widened to complex, a
// length-n complex DFT runs, and the half spectrum (or real part) is kept.
// The inverse is the sign +1 transform, by conjugation like complex plans.
//
// One real dimension d (is, os in the units of each side) over vector loops V,
// from buffer src (offset in complex elements) to dst; `same_buf` when src and
// dst are one buffer (in place).
static int plan_real_line(Builder &b, bool fwd, Dim d, const std::vector<Dim> &V, int src,
                          int64_t src_off, int dst, int64_t dst_off, bool same_buf)
{
    PlanImpl *p = b.p;
    const int prec = p->prob.prec;
    const int eb = elem_bytes(prec);
    const int64_t n = d.n;
    int64_t H = 1;
    for (const Dim &v : V) H *= v.n;
    bool pack = n % 2 == 0 && (fwd ? d.is == 1 : d.os == 1);
    for (const Dim &v : V) pack &= (fwd ? v.is : v.os) % 2 == 0;
    if (pack) {
        const int64_t h = n / 2;
        void *tw = table_alloc(p, (size_t)(h / 2 + 1) * eb);
        if (!tw) return fail(MFFT_ENOMEM, "twiddle table allocation failed");
        hipError_t e = launch_gen_roots(tw, prec, h / 2 + 1, n, p->stream);
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("twiddle kernel: ") + hipGetErrorString(e));
        // the real side viewed as complex: vector strides halve
        std::vector<Dim> Vc = V;
        for (Dim &v : Vc) (fwd ? v.is : v.os) /= 2;
        // one pass when the half-length transform is a specialized leaf: the
        // split (or combine) runs in its store (load) through LDS.  In place
        // only when each real row starts where its complex row does.
        bool same_rows = true;
        for (const Dim &v : V) same_rows &= fwd ? v.is == 2 * v.os : v.os == 2 * v.is;
        // (the fused split and combine exist for half-lengths up to 4096)
        if (leaf_supported(prec, h) && h <= 4096 && (fwd ? d.os == 1 : d.is == 1) &&
            (!same_buf || same_rows)) {
            const size_t before = p->passes.size();
            const int64_t top = b.scratch_top, hi = b.scratch_hi;
            int rc = plan_line(b, Dim{h, 1, 1}, Vc, src, dst, src_off, dst_off, !fwd, !fwd);
            if (rc) return rc;
            if (p->passes.size() == before + 1 && p->passes.back().kernel == 1) {
                Pass &ps = p->passes.back();
                ps.a.flags |= fwd ? PF_R2C : PF_C2R;
                ps.a.post = tw;
                if (!fwd) ps.variant &= ~1;   // the combine replaces the prefetch
                ps.desc += fwd ? " +split" : " +combine";
                return MFFT_OK;
            }
            p->passes.resize(before);
            b.scratch_top = top;
            b.scratch_hi = hi;
        }
        const int64_t off = b.scratch_take(H * h * eb) / eb;
        if (fwd) {
            int zsrc = src;
            int64_t zoff = src_off;
            std::vector<Dim> Vu = packed(V, h, 0);   // untangle reads packed Z
            if (h > 1) {
                int rc = plan_line(b, Dim{h, 1, 1}, packed(Vc, h, 1), src, BUF_SCRATCH, src_off, off,
                                   false, false);
                if (rc) return rc;
                zsrc = BUF_SCRATCH;
                zoff = off;
            } else {
                for (size_t i = 0; i < Vu.size(); ++i) Vu[i].is = Vc[i].is;
            }
            return add_real_pass(b, RK_UNTANGLE, n, h / 2 + 1, 1, d.os, Vu, zsrc, zoff, dst, dst_off,
                                 tw, "untangle");
        }
        int rc = add_real_pass(b, RK_TANGLE, n, h / 2 + 1, d.is, 1, packed(V, h, 1), src, src_off,
                               BUF_SCRATCH, off, tw, "tangle");
        if (rc) return rc;
        std::vector<Dim> Vi = packed(Vc, h, 0);
        if (h > 1) return plan_line(b, Dim{h, 1, 1}, Vi, BUF_SCRATCH, dst, off, dst_off, true, true);
        std::vector<Dim> all = Vi;
        all.push_back({1, 1, 1});
        return add_copy_pass(b, all, BUF_SCRATCH, dst, off, dst_off, "copy");
    }
    const int64_t o0 = b.scratch_take(H * n * eb) / eb;
    const int64_t o1 = n > 1 ? b.scratch_take(H * n * eb) / eb : o0;
    std::vector<Dim> Vp = packed(packed(V, n, 0), n, 1);
    if (fwd) {
        int rc = add_real_pass(b, RK_WIDEN, n, n, d.is, 1, packed(V, n, 1), src, src_off,
                               BUF_SCRATCH, o0, nullptr, "widen");
        if (rc) return rc;
        if (n > 1) {
            rc = plan_line(b, Dim{n, 1, 1}, Vp, BUF_SCRATCH, BUF_SCRATCH, o0, o1, false, false);
            if (rc) return rc;
        }
        std::vector<Dim> all = packed(V, n, 0);
        all.push_back({n / 2 + 1, 1, d.os});
        return add_copy_pass(b, all, BUF_SCRATCH, dst, o1, dst_off, "half spectrum");
    }
    int rc = add_real_pass(b, RK_HERM, n, n, d.is, 1, packed(V, n, 1), src, src_off, BUF_SCRATCH,
                           o0, nullptr, "symmetric extension");
    if (rc) return rc;
    if (n > 1) {
        rc = plan_line(b, Dim{n, 1, 1}, Vp, BUF_SCRATCH, BUF_SCRATCH, o0, o1, true, true);
        if (rc) return rc;
    }
    return add_real_pass(b, RK_REAL, n, n, 1, d.os, packed(V, n, 0), BUF_SCRATCH, o1, dst, dst_off,
                         nullptr, "real part");
}

// MFFT_NO_SCRATCH: a plan that still needs scratch has no form without it.
static int no_scratch_check(const PlanImpl *p)
{
    if ((p->flags & MFFT_NO_SCRATCH) && p->scratch_bytes)
        return fail(MFFT_ENOTSUP, "no plan without scratch memory for this problem");
    return MFFT_OK;
}

// Rank-r real transforms (the last dimension is the halved one): forward, the
// real step along the last dimension (the others join the vector loops), then
// complex steps along the others in place on the output; inverse, complex
// steps along the others from the input into packed scratch (the input is
// not modified), then the real step into the output.
static int build_real_plan(PlanImpl *p)
{
    Builder b;
    b.p = p;
    const Problem &pr = p->prob;
    p->passes.clear();
    if (pr.empty) return MFFT_OK;
    const int eb = elem_bytes(pr.prec);
    const bool fwd = pr.kind == 1;
    const int dst = pr.inplace ? BUF_IN : BUF_OUT;
    const Dim d = pr.N.back();
    const int64_t hc = d.n / 2 + 1;   // complex points along the halved dimension
    std::vector<Dim> others(pr.N.begin(), pr.N.end() - 1);
    std::vector<Dim> V1 = pr.V;
    V1.insert(V1.end(), others.begin(), others.end());
    int rc = MFFT_OK;
    if (fwd) {
        rc = plan_real_line(b, true, d, V1, BUF_IN, 0, dst, 0, pr.inplace);
        for (size_t j = 0; j < others.size() && rc == MFFT_OK; ++j) {
            std::vector<Dim> Vj = copy_o(pr.V);
            for (size_t k = 0; k < others.size(); ++k)
                if (k != j) Vj.push_back({others[k].n, others[k].os, others[k].os});
            Vj.push_back({hc, d.os, d.os});
            rc = plan_line(b, Dim{others[j].n, others[j].os, others[j].os}, Vj, dst, dst, 0, 0,
                           false, false);
        }
    } else if (others.empty()) {
        rc = plan_real_line(b, false, d, pr.V, BUF_IN, 0, dst, 0, pr.inplace);
    } else {
        // complex half-spectrum tensor in packed scratch: [V..., others..., hc]
        std::vector<Dim> all = pr.V;
        all.insert(all.end(), others.begin(), others.end());
        all.push_back({hc, d.is, d.is});
        const std::vector<Dim> pk = packed(all, 1, 1);   // os: packed strides
        int64_t total = 1;
        for (const Dim &x : all) total *= x.n;
        const int64_t S = b.scratch_take(total * eb) / eb;
        const size_t nv = pr.V.size();
        for (size_t j = 0; j < others.size() && rc == MFFT_OK; ++j) {
            const bool first = j == 0;
            std::vector<Dim> Vj;
            for (size_t i = 0; i < all.size(); ++i) {
                if (i == nv + j) continue;
                const int64_t is = first ? all[i].is : pk[i].os;
                Vj.push_back({all[i].n, is, pk[i].os});
            }
            const Dim dj{others[j].n, first ? others[j].is : pk[nv + j].os, pk[nv + j].os};
            rc = plan_line(b, dj, Vj, first ? BUF_IN : BUF_SCRATCH, BUF_SCRATCH, first ? 0 : S, S,
                           true, true);
        }
        if (rc == MFFT_OK) {
            // the real step reads the packed scratch, writes the user's layout
            std::vector<Dim> Vr;
            for (size_t i = 0; i + 1 < all.size(); ++i) {
                const Dim &u = i < nv ? pr.V[i] : others[i - nv];
                Vr.push_back({u.n, pk[i].os, u.os});
            }
            rc = plan_real_line(b, false, Dim{d.n, 1, d.os}, Vr, BUF_SCRATCH, S, dst, 0, false);
        }
    }
    if (rc) return rc;
    p->scratch_bytes = (size_t)b.scratch_hi;
    return no_scratch_check(p);
}

int build_plan(PlanImpl *p)
{
    if (p->prob.kind != 0) return build_real_plan(p);
    Builder b;
    b.p = p;
    const Problem &pr = p->prob;
    p->passes.clear();
    if (pr.empty) return MFFT_OK;
    const bool conj = pr.sign > 0;
    const int eb = elem_bytes(pr.prec);

    std::vector<Dim> N = pr.N, V = pr.V;
    int src = BUF_IN;
    int64_t src_off = 0;
    const int dst = pr.inplace ? BUF_IN : BUF_OUT;

    bool same_layout = true;
    for (const Dim &d : N) same_layout &= d.is == d.os;
    for (const Dim &d : V) same_layout &= d.is == d.os;

    if (N.empty()) {
        if (pr.inplace && same_layout) return MFFT_OK;   // copy onto itself
        std::vector<Dim> all = V;
        if (pr.inplace && (p->flags & MFFT_NO_SCRATCH)) {
            int rc = plan_rank0_transpose_inplace(b, V);
            if (rc) return rc;
            p->scratch_bytes = 0;
            return MFFT_OK;
        }
        if (pr.inplace) {
            const int64_t off = b.scratch_take(pr.howmany * eb) / eb;
            int rc = add_copy_pass(b, packed(all, 1, 1), BUF_IN, BUF_SCRATCH, 0, off, "snapshot");
            if (rc) return rc;
            rc = add_copy_pass(b, packed(all, 1, 0), BUF_SCRATCH, dst, off, 0, "copy");
            if (rc) return rc;
        } else {
            int rc = add_copy_pass(b, all, BUF_IN, BUF_OUT, 0, 0, "copy");
            if (rc) return rc;
        }
        p->scratch_bytes = (size_t)b.scratch_hi;
        return no_scratch_check(p);
    }

    int64_t persistent = 0;
    if (pr.inplace && !same_layout) {
        // read the input before anything is written: copy it to packed scratch
        std::vector<Dim> all = V;
        all.insert(all.end(), N.begin(), N.end());
        const int64_t total = pr.howmany * pr.n_total;
        const int64_t off = b.scratch_take(total * eb) / eb;
        int rc = add_copy_pass(b, packed(all, 1, 1), BUF_IN, BUF_SCRATCH, 0, off, "snapshot");
        if (rc) return rc;
        std::vector<Dim> pk = packed(all, 1, 1);
        for (size_t i = 0; i < V.size(); ++i) V[i].is = pk[i].os;
        for (size_t i = 0; i < N.size(); ++i) N[i].is = pk[V.size() + i].os;
        src = BUF_SCRATCH;
        src_off = off;
        persistent = b.scratch_top;
    }

    // first dimension: smallest input stride (unit-stride rows load best)
    std::vector<int> order(N.size());
    for (size_t i = 0; i < N.size(); ++i) order[i] = (int)i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return std::llabs(N[x].is) < std::llabs(N[y].is);
    });
    for (size_t step = 0; step < order.size(); ++step) {
        const int j = order[step];
        b.scratch_top = persistent;
        std::vector<Dim> Vs;
        Dim d = N[j];
        if (step == 0) {
            Vs = V;
            for (size_t i = 0; i < N.size(); ++i)
                if ((int)i != j) Vs.push_back(N[i]);
            int rc = plan_line(b, d, Vs, src, dst, src_off, 0, conj, conj);
            if (rc) return rc;
        } else {
            Vs = copy_o(V);
            for (size_t i = 0; i < N.size(); ++i)
                if ((int)i != j) Vs.push_back({N[i].n, N[i].os, N[i].os});
            d = {d.n, d.os, d.os};
            int rc = plan_line(b, d, Vs, dst, dst, 0, 0, conj, conj);
            if (rc) return rc;
        }
    }
    p->scratch_bytes = (size_t)b.scratch_hi;
    return no_scratch_check(p);
}

// ------------------------------------------------------------ execution

static char *resolve_buf(const PlanImpl *p, int id, int64_t off, const void *in, void *out,
                         void *scratch)
{
    const int eb = elem_bytes(p->prob.prec);
    char *base = id == BUF_IN ? (char *)in : id == BUF_OUT ? (char *)out : (char *)scratch;
    return base + off * eb;
}

PassArgs resolve_pass(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch)
{
    PassArgs a = ps.a;
    a.in = resolve_buf(p, ps.src, ps.src_off, in, out, scratch);
    a.out = resolve_buf(p, ps.dst, ps.dst_off, in, out, scratch);
    if (ps.aux_off >= 0) a.aux = (char *)scratch + ps.aux_off;
    return a;
}

CopyArgs resolve_copy(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch)
{
    CopyArgs c = ps.c;
    c.in = resolve_buf(p, ps.src, ps.src_off, in, out, scratch);
    c.out = resolve_buf(p, ps.dst, ps.dst_off, in, out, scratch);
    return c;
}

RealArgs resolve_real(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch)
{
    RealArgs r = ps.r;
    r.in = resolve_buf(p, ps.src, ps.src_off, in, out, scratch);
    r.out = resolve_buf(p, ps.dst, ps.dst_off, in, out, scratch);
    return r;
}

TransposeArgs resolve_transpose(const PlanImpl *p, const Pass &ps, const void *in, void *out,
                                void *scratch)
{
    TransposeArgs t = ps.t;
    t.data = resolve_buf(p, ps.dst, ps.dst_off, in, out, scratch);
    return t;
}

PermuteArgs resolve_permute(const PlanImpl *p, const Pass &ps, const void *in, void *out,
                            void *scratch)
{
    PermuteArgs a = ps.pm;
    a.data = resolve_buf(p, ps.dst, ps.dst_off, in, out, scratch);
    return a;
}

size_t generic_lds_bytes(const Pass &ps)
{
    return tile_lds_bytes(ps.a.n, ps.a.bt, ps.prec, ps.emax);
}

int run_plan(const PlanImpl *p, const void *in, void *out, void *scratch, hipStream_t s)
{
    for (const Pass &ps : p->passes) {
        hipError_t e;
        if (ps.kind == 1) {
            e = launch_copy(resolve_copy(p, ps, in, out, scratch), s);
        } else if (ps.kind == 2) {
            e = launch_real(resolve_real(p, ps, in, out, scratch), p->prob.prec, s);
        } else if (ps.kind == 3) {
            e = launch_transpose_sq(resolve_transpose(p, ps, in, out, scratch), s);
        } else if (ps.kind == 4) {
            e = launch_permute_items(resolve_permute(p, ps, in, out, scratch), s);
        } else {
            const PassArgs a = resolve_pass(p, ps, in, out, scratch);
            if (ps.kernel == 1)
                e = launch_leaf(a, p->prob.prec, a.n, ps.variant, (int)ps.grid, s);
            else
                e = launch_pass(a, p->prob.prec, ps.emax, ps.lds_bytes, s);
        }
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("launch: ") + hipGetErrorString(e));
    }
    return MFFT_OK;
}

}  // namespace mfft
