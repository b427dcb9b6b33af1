// C ABI: plan / execute / destroy, plan info, wisdom, errors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "plan.h"

namespace mfft {

const char *last_error_text();
extern size_t g_lds_budget;
extern int g_num_cus;

static std::mutex g_plan_mutex;
static bool g_inited = false;
static std::string g_arch = "unknown";

// Scratch of mfft_execute_static_scratch: a fixed device array the loader
// places on every GPU the library runs on, held until the process ends, so
// that executing a plan that needs scratch allocates nothing.  In host code
// `scratch` names a host-side stand-in; the device address comes from
// hipGetSymbolAddress, resolved once per device and kept in g_static_ptr.
static __device__ __align__(256) unsigned char scratch[MFFT_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_static_mutex;
static void *g_static_ptr[kMaxDevices];

// Device address of `scratch` on device `dev` (which must be current).
static int static_scratch_ptr(int dev, void **ptr)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(MFFT_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_static_mutex);
    if (!g_static_ptr[dev]) {
        void *q = nullptr;
        hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return fail(MFFT_EHIP, std::string("static scratch address: ") + hipGetErrorString(e));
        g_static_ptr[dev] = q;
    }
    *ptr = g_static_ptr[dev];
    return MFFT_OK;
}

static int init_device()
{
    if (g_inited) return MFFT_OK;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MFFT_EHIP, std::string("no HIP device: ") + hipGetErrorString(e));
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return fail(MFFT_EHIP, hipGetErrorString(e));
    g_arch = prop.gcnArchName;
    size_t lds = prop.sharedMemPerBlock;
    if (const char *env = getenv("MFFT_LDS_BUDGET")) lds = std::min(lds, (size_t)atol(env));
    // keep a little LDS for the batched kernel's static variables
    g_lds_budget = std::min<size_t>(lds, 163840) - 256;
    g_num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    void *q = nullptr;
    int rc = static_scratch_ptr(dev, &q);
    if (rc) return rc;
    g_inited = true;
    return MFFT_OK;
}

const std::string &device_arch() { return g_arch; }

// ------------------------------------------------------------ wisdom store

static std::mutex g_wisdom_mutex;
static std::map<std::string, std::string> g_wisdom;

bool wisdom_lookup(const std::string &key, std::string *val)
{
    std::lock_guard<std::mutex> lk(g_wisdom_mutex);
    auto it = g_wisdom.find(key);
    if (it == g_wisdom.end()) return false;
    *val = it->second;
    return true;
}

void wisdom_record(const std::string &key, const std::string &val)
{
    std::lock_guard<std::mutex> lk(g_wisdom_mutex);
    g_wisdom[key] = val;
}

static void destroy_impl(PlanImpl *p)
{
    for (DeviceAlloc &d : p->tables) dev_free(p, d.ptr, d.bytes);
    p->tables.clear();
    if (p->scratch) dev_free(p, p->scratch, p->scratch_bytes);
    p->scratch = nullptr;
}

int rebuild_plan(PlanImpl *p)
{
    // table kernels of the previous build may still be queued
    (void)hipStreamSynchronize(p->stream);
    destroy_impl(p);
    p->table_bytes = 0;
    p->scratch_bytes = 0;
    p->passes.clear();
    return build_plan(p);
}

// Wisdom key of the structural choice for lines of one length (shared by
// every problem with such lines, whatever its strides and vector loops).
static std::string length_key(const PlanImpl *p, int64_t n, unsigned flags)
{
    return std::string("line c") + (p->prob.prec ? "64" : "32") + " n=" + std::to_string(n) + " " +
           g_arch + ((flags & MFFT_NO_SCRATCH) ? " noscratch" : "");
}

// Stored choices for the problem: the problem's own entry (structure and
// kernel variants), else one entry per transform length (structure).  True
// when the plan is fully determined by them.
static int apply_wisdom(PlanImpl *p, const std::string &key, unsigned flags, bool *found)
{
    *found = false;
    std::string val;
    if (wisdom_lookup(key, &val)) {
        const size_t bar = val.find('|');
        std::map<int64_t, StructChoice> st;
        if (parse_structure(bar == std::string::npos ? "-" : val.substr(0, bar), &st)) {
            int rc = MFFT_OK;
            if (!st.empty()) {
                p->overrides = st;
                rc = rebuild_plan(p);
                if (rc) return rc;
            }
            if (apply_choices(p, val)) {
                *found = true;
                return MFFT_OK;
            }
        }
    }
    if (p->prob.kind != 0) return MFFT_OK;
    bool all = true;
    std::map<int64_t, StructChoice> st;
    for (const Dim &d : p->prob.N) {
        int64_t n = 0;
        StructChoice c;
        if (wisdom_lookup(length_key(p, d.n, flags), &val) && parse_choice(val, &n, &c) && n == d.n) {
            if (!c.empty()) st[d.n] = c;
        } else {
            all = false;
        }
    }
    if (!st.empty()) {
        p->overrides = st;
        int rc = rebuild_plan(p);
        if (rc) return rc;
    }
    *found = all;
    return MFFT_OK;
}

// Plan without the global lock (used for the FP64 sub-transforms that build
// Rader and Bluestein spectra while another plan is being made).
int plan_internal(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                  const mfft_iodim *hdims, int inplace, int sign, int prec, hipStream_t stream,
                  unsigned flags, const mfft_allocator *alloc, int kind)
{
    *out = nullptr;
    int rc = init_device();
    if (rc) return rc;
    mfft_plan pl = new (std::nothrow) mfft_plan_s();
    if (!pl) return fail(MFFT_ENOMEM, "host allocation failed");
    PlanImpl *p = &pl->impl;
    rc = kind ? canonicalize_real(kind, rank, dims, howmany_rank, hdims, inplace, prec, &p->prob)
              : canonicalize(rank, dims, howmany_rank, hdims, inplace, sign, prec, &p->prob);
    if (rc) {
        delete pl;
        return rc;
    }
    p->flags = flags;
    p->stream = stream;
    if (alloc) {
        p->alloc = *alloc;
        p->has_alloc = true;
    }
    (void)hipGetDevice(&p->device);
    rc = build_plan(p);
    if (rc == MFFT_OK && !p->prob.empty) {
        // wisdom (stored choices) first, then measurement, else estimate defaults
        // plans without scratch have other passes: their own wisdom entries
        const std::string key = problem_key(p->prob) + " " + g_arch +
                                ((flags & MFFT_NO_SCRATCH) ? " noscratch" : "");
        const bool use_wisdom = !(flags & MFFT_NO_WISDOM);
        bool found = false;
        if (use_wisdom) rc = apply_wisdom(p, key, flags, &found);
        if (rc) {
            // a stored choice that no longer plans: fall back to the estimate
            p->overrides.clear();
            rc = rebuild_plan(p);
            found = false;
        }
        if (rc == MFFT_OK) {
            if (found) {
                p->from_wisdom = true;
            } else if (flags & MFFT_WISDOM_ONLY) {
                rc = fail(MFFT_ENOWISDOM, "no stored plan for " + key);
            } else if (flags & MFFT_MEASURE) {
                rc = measure_structure(p);
                if (rc == MFFT_OK) rc = measure_plan(p);
                if (rc == MFFT_OK && use_wisdom) {
                    wisdom_record(key, plan_choices(p));
                    if (p->prob.kind == 0)
                        for (const Dim &d : p->prob.N) {
                            auto it = p->overrides.find(d.n);
                            wisdom_record(length_key(p, d.n, flags),
                                          choice_text(d.n, it == p->overrides.end()
                                                               ? StructChoice{}
                                                               : it->second));
                        }
                }
            }
        }
    }
    if (rc == MFFT_OK && p->scratch_bytes && !(flags & kPlanNoOwnScratch)) {
        p->scratch = dev_alloc(p, p->scratch_bytes);
        if (!p->scratch) rc = fail(MFFT_ENOMEM, "scratch allocation failed");
    }
    if (rc == MFFT_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = fail(MFFT_EHIP, std::string("table generation: ") + hipGetErrorString(e));
    }
    if (rc) {
        // table kernels may still run on the stream: let them finish before
        // their memory goes back to the allocator
        (void)hipStreamSynchronize(stream);
        destroy_impl(p);
        delete pl;
        return rc;
    }
    std::ostringstream d;
    d << problem_key(p->prob) << "\n";
    p->bytes_passes = 0;
    for (const Pass &ps : p->passes) {
        d << "  " << ps.desc;
        if (ps.kernel == 1)
            d << " [leaf kernel"
              << ((ps.a.flags & PF_LEAF_COL)  ? " columns"
                  : (ps.a.flags & PF_LEAF_CR) ? " columns->rows"
                  : (ps.a.flags & PF_LEAF_RC) ? " rows->columns"
                                              : "")
              << " v"
              << ps.variant << (ps.persistent ? " persistent" : "") << " grid=" << ps.grid
              << "]";
        d << "\n";
        p->bytes_passes += ps.bytes;
    }
    if (p->from_wisdom) d << "  (choices from wisdom)\n";
    p->desc = d.str();
    *out = pl;
    return MFFT_OK;
}

int plan_dft_locked(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                    const mfft_iodim *hdims, int inplace, int sign, int prec, unsigned flags,
                    const mfft_allocator *alloc, hipStream_t stream)
{
    std::lock_guard<std::mutex> lk(g_plan_mutex);
    return plan_internal(out, rank, dims, howmany_rank, hdims, inplace, sign, prec, stream, flags,
                         alloc);
}

}  // namespace mfft

using namespace mfft;

extern "C" {

const char *mfft_last_error(void) { return last_error_text(); }

const char *mfft_version(void) { return "mfft 0.1.0 (gfx950)"; }

static int check_flags(unsigned flags, mfft_prec prec)
{
    const unsigned known = MFFT_MEASURE | MFFT_WISDOM_ONLY | MFFT_NO_WISDOM | MFFT_FP32_TWIDDLES |
                           MFFT_NO_SCRATCH;
    if (flags & ~known) return fail(MFFT_EINVAL, "unknown planner flag bits");
    if ((flags & MFFT_FP32_TWIDDLES) && prec != MFFT_C32)
        return fail(MFFT_EINVAL, "MFFT_FP32_TWIDDLES applies to MFFT_C32 plans only");
    return MFFT_OK;
}

int mfft_plan_dft(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                  const mfft_iodim *howmany_dims, int inplace, int sign, mfft_prec prec,
                  unsigned flags, const mfft_allocator *alloc, void *hip_stream)
{
    if (!out) return fail(MFFT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_flags(flags, prec);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mutex);
    return plan_internal(out, rank, dims, howmany_rank, howmany_dims, inplace, sign, (int)prec,
                         (hipStream_t)hip_stream, flags, alloc);
}

int mfft_plan_dft_r2c(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *howmany_dims, int inplace, mfft_prec prec, unsigned flags,
                      const mfft_allocator *alloc, void *hip_stream)
{
    if (!out) return fail(MFFT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_flags(flags, prec);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mutex);
    return plan_internal(out, rank, dims, howmany_rank, howmany_dims, inplace, -1, (int)prec,
                         (hipStream_t)hip_stream, flags, alloc, 1);
}

int mfft_plan_dft_c2r(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *howmany_dims, int inplace, mfft_prec prec, unsigned flags,
                      const mfft_allocator *alloc, void *hip_stream)
{
    if (!out) return fail(MFFT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_flags(flags, prec);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_plan_mutex);
    return plan_internal(out, rank, dims, howmany_rank, howmany_dims, inplace, 1, (int)prec,
                         (hipStream_t)hip_stream, flags, alloc, 2);
}

int mfft_execute_scratch(mfft_plan plan, const void *in, void *out, void *scratch,
                         void *hip_stream)
{
    if (!plan) return fail(MFFT_EINVAL, "plan is NULL");
    const PlanImpl *p = &plan->impl;
    if (p->prob.empty) return MFFT_OK;
    const size_t eb = p->prob.prec ? 16 : 8;
    if (!in || !out) return fail(MFFT_EINVAL, "NULL data pointer");
    if (((uintptr_t)in % eb) || ((uintptr_t)out % eb))
        return fail(MFFT_EALIGN, "data pointers must be aligned to the complex element size");
    if (p->prob.inplace && in != out)
        return fail(MFFT_EALIGN, "in-place plan executed with in != out");
    if (!p->prob.inplace && in == out)
        return fail(MFFT_EALIGN, "out-of-place plan executed with in == out");
    if (p->scratch_bytes && !scratch) return fail(MFFT_EINVAL, "plan needs scratch memory");
    return run_plan(p, in, out, scratch, (hipStream_t)hip_stream);
}

int mfft_execute(mfft_plan plan, const void *in, void *out, void *hip_stream)
{
    if (!plan) return fail(MFFT_EINVAL, "plan is NULL");
    return mfft_execute_scratch(plan, in, out, plan->impl.scratch, hip_stream);
}

int mfft_execute_static_scratch(mfft_plan plan, const void *in, void *out, void *hip_stream)
{
    if (!plan) return fail(MFFT_EINVAL, "plan is NULL");
    const PlanImpl *p = &plan->impl;
    if (p->scratch_bytes > MFFT_STATIC_SCRATCH_BYTES)
        return fail(MFFT_ENOMEM, "plan needs " + std::to_string(p->scratch_bytes) +
                                     " bytes of scratch; the static scratch holds " +
                                     std::to_string((size_t)MFFT_STATIC_SCRATCH_BYTES));
    void *s = nullptr;
    if (p->scratch_bytes) {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return fail(MFFT_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
        int rc = static_scratch_ptr(dev, &s);
        if (rc) return rc;
    }
    return mfft_execute_scratch(plan, in, out, s, hip_stream);
}

int mfft_plan_info(mfft_plan plan, mfft_plan_info_t *info)
{
    if (!plan || !info) return fail(MFFT_EINVAL, "NULL argument");
    const PlanImpl *p = &plan->impl;
    std::memset(info, 0, sizeof(*info));
    info->prec = p->prob.prec;
    info->sign = p->prob.sign;
    info->rank = (int)p->prob.N.size();
    info->howmany_rank = (int)p->prob.V.size();
    info->inplace = p->prob.inplace;
    info->n_passes = (int)p->passes.size();
    info->n_total = p->prob.empty ? 0 : p->prob.n_total;
    info->howmany = p->prob.empty ? 0 : p->prob.howmany;
    const double N = (double)info->n_total;
    const double eb = p->prob.prec ? 16.0 : 8.0;
    info->flops = N > 1 ? 5.0 * N * std::log2(N) * (double)info->howmany : 0.0;
    info->bytes_compulsory = 2.0 * eb * N * (double)info->howmany;
    if (p->prob.kind != 0) {
        // real data: half the nominal flops; n reals one way, n/2+1 complex the other
        info->flops *= 0.5;
        const int64_t nl = p->prob.N.back().n;
        info->bytes_compulsory =
            (eb / 2 * N + eb * N / (double)nl * (double)(nl / 2 + 1)) * (double)info->howmany;
    }
    info->bytes_passes = p->bytes_passes;
    info->scratch_bytes = p->scratch_bytes;
    info->table_bytes = p->table_bytes;
    std::strncpy(info->desc, p->desc.c_str(), sizeof(info->desc) - 1);
    auto put = [&](int r) {
        if (info->n_radices < MFFT_INFO_RADICES) info->radices[info->n_radices++] = r;
    };
    for (const Pass &ps : p->passes) {
        if (ps.kind == 0) {
            if (ps.kernel == 1) {
                // the specialized leaf kernel runs its own sequence
                for (int s = 0; s < leaf_radix_count(ps.a.n); ++s) put(leaf_radix_at(ps.a.n, s));
            } else {
                for (int s = 0; s < ps.a.nst; ++s) put(ps.a.st[s].R);
            }
        }
        put(0);
    }
    return MFFT_OK;
}

int mfft_plan_destroy(mfft_plan plan)
{
    if (!plan) return MFFT_OK;
    destroy_impl(&plan->impl);
    delete plan;
    return MFFT_OK;
}

int mfft_wisdom_export(char **buf, size_t *len)
{
    if (!buf || !len) return fail(MFFT_EINVAL, "NULL argument");
    std::ostringstream s;
    s << "mfft-wisdom 1 " << mfft_version() << "\n";
    {
        std::lock_guard<std::mutex> lk(g_wisdom_mutex);
        for (auto &kv : g_wisdom) s << kv.first << " => " << kv.second << "\n";
    }
    const std::string t = s.str();
    char *m = (char *)std::malloc(t.size() + 1);
    if (!m) return fail(MFFT_ENOMEM, "host allocation failed");
    std::memcpy(m, t.c_str(), t.size() + 1);
    *buf = m;
    *len = t.size();
    return MFFT_OK;
}

int mfft_wisdom_import(const char *buf, size_t len)
{
    if (!buf) return fail(MFFT_EINVAL, "NULL buffer");
    std::istringstream s(std::string(buf, len));
    std::string line;
    if (!std::getline(s, line) || line.rfind("mfft-wisdom 1 ", 0) != 0)
        return fail(MFFT_EINVAL, "not mfft wisdom text");
    std::map<std::string, std::string> add;
    while (std::getline(s, line)) {
        if (line.empty()) continue;
        const size_t k = line.find(" => ");
        if (k == std::string::npos) return fail(MFFT_EINVAL, "malformed wisdom line");
        add[line.substr(0, k)] = line.substr(k + 4);
    }
    std::lock_guard<std::mutex> lk(g_wisdom_mutex);
    for (auto &kv : add) g_wisdom[kv.first] = kv.second;
    return MFFT_OK;
}

int mfft_wisdom_forget(void)
{
    std::lock_guard<std::mutex> lk(g_wisdom_mutex);
    g_wisdom.clear();
    return MFFT_OK;
}

void mfft_free(void *p) { std::free(p); }

}  // extern "C"
