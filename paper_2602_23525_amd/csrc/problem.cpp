// Problem validation and canonicalization (host only, no HIP calls).
//
// The problem is dft(N, V, I, O) of Section 4.1: N and V are I/O tensors,
// i.e. sets of I/O dimensions (n, is, os).  Canonical form:
//   - a length-0 dimension anywhere makes the whole problem an empty loop;
//   - length-1 dimensions are dropped (a size-1 DFT is a copy, Section 4.1);
//   - vector loops that address memory as one longer loop are merged
//     (the loop order is unspecified, so V can be reordered freely);
//   - two (vector, frequency) index pairs writing one output address are
//     rejected, since the result would depend on the loop order.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <sstream>
#include <string>
#include <unordered_set>

#include "plan.h"

namespace mfft {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

const char *last_error_text() { return g_last_error.c_str(); }

static bool mul_overflows(int64_t a, int64_t b)
{
    __int128 p = (__int128)a * (__int128)b;
    return p > (__int128)INT64_MAX / 4 || p < -(__int128)INT64_MAX / 4;
}

// Is v a sum of delta_j * |os_j| over the first k of the dims d (sorted by
// |os|), |delta_j| < n_j?  span[i] is the largest such sum over the first i
// dims.  Counts visited nodes against *budget (false once it runs out, with
// *budget < 0).
static bool in_difference_set(const std::vector<Dim> &d, const std::vector<int64_t> &span,
                              size_t k, int64_t v, int64_t *budget)
{
    if (v == 0) return true;
    if (k == 0 || --*budget < 0) return false;
    const int64_t o = std::llabs(d[k - 1].os), m = d[k - 1].n - 1, s = span[k - 1];
    if (std::llabs(v) > s + m * o) return false;
    // delta * o within s of v
    auto fdiv = [](int64_t a, int64_t q) { return a / q - ((a % q != 0) && ((a < 0) != (q < 0))); };
    const int64_t lo = std::max(-m, -fdiv(-(v - s), o)), hi = std::min(m, fdiv(v + s, o));
    for (int64_t delta = lo; delta <= hi; ++delta) {
        if (in_difference_set(d, span, k - 1, v - delta * o, budget)) return true;
        if (*budget < 0) return false;
    }
    return false;
}

// Injectivity of the output map over all dims with n > 1.  Two index tuples
// collide exactly when some nonzero (delta_j), |delta_j| < n_j, has
// sum delta_j * os_j = 0; taking the dim of largest |os| with delta_j != 0 as
// the last, its multiple delta_k * |os_k| must be a difference of outputs of
// the dims of smaller |os|, which only happens when it is at most their span
// (so a layout where each |os| exceeds the span of the smaller ones is
// injective at once).  Otherwise the multiples below that span are decided by
// a bounded search over the smaller dims; past its budget, an enumeration of
// every output for problems of at most 2^22 elements, else refused.
static bool outputs_injective(const std::vector<Dim> &all)
{
    std::vector<Dim> d;
    for (const Dim &x : all)
        if (x.n > 1) {
            if (x.os == 0) return false;
            d.push_back(x);
        }
    std::sort(d.begin(), d.end(),
              [](const Dim &a, const Dim &b) { return std::llabs(a.os) < std::llabs(b.os); });
    std::vector<int64_t> span(d.size() + 1, 0);
    for (size_t i = 0; i < d.size(); ++i) span[i + 1] = span[i] + (d[i].n - 1) * std::llabs(d[i].os);
    int64_t budget = (int64_t)1 << 24;
    bool decided = true;
    for (size_t k = 1; k < d.size() && decided; ++k) {
        const int64_t o = std::llabs(d[k].os);
        for (int64_t delta = 1; delta < d[k].n && delta * o <= span[k]; ++delta) {
            if (in_difference_set(d, span, k, delta * o, &budget)) return false;
            if (budget < 0) {
                decided = false;
                break;
            }
        }
    }
    if (decided) return true;
    int64_t total = 1;
    for (const Dim &x : d) {
        total *= x.n;
        if (total > (1 << 22)) return false;
    }
    std::unordered_set<int64_t> seen;
    seen.reserve((size_t)total * 2);
    std::vector<int64_t> idx(d.size(), 0);
    for (int64_t i = 0; i < total; ++i) {
        int64_t off = 0;
        for (size_t j = 0; j < d.size(); ++j) off += idx[j] * d[j].os;
        if (!seen.insert(off).second) return false;
        for (size_t j = 0; j < d.size(); ++j) {
            if (++idx[j] < d[j].n) break;
            idx[j] = 0;
        }
    }
    return true;
}

int canonicalize(int rank, const mfft_iodim *dims, int howmany_rank, const mfft_iodim *hdims,
                 int inplace, int sign, int prec, Problem *out)
{
    Problem p;
    if (rank < 0 || rank > 8) return fail(MFFT_EINVAL, "rank must be in [0, 8]");
    if (howmany_rank < 0 || howmany_rank > 8)
        return fail(MFFT_EINVAL, "howmany_rank must be in [0, 8]");
    if (rank > 0 && !dims) return fail(MFFT_EINVAL, "dims is NULL");
    if (howmany_rank > 0 && !hdims) return fail(MFFT_EINVAL, "howmany_dims is NULL");
    if (sign != -1 && sign != 1) return fail(MFFT_EINVAL, "sign must be -1 or +1");
    if (prec != MFFT_C32 && prec != MFFT_C64) return fail(MFFT_EINVAL, "unknown precision");
    if (inplace != 0 && inplace != 1) return fail(MFFT_EINVAL, "inplace must be 0 or 1");
    p.sign = sign;
    p.prec = prec;
    p.inplace = inplace != 0;

    std::vector<Dim> N, V;
    int64_t ext_in = 0, ext_out = 0;
    for (int i = 0; i < rank + howmany_rank; ++i) {
        const mfft_iodim &d = i < rank ? dims[i] : hdims[i - rank];
        if (d.n < 0) return fail(MFFT_EINVAL, "negative length");
        if (d.n > ((int64_t)1 << 40)) return fail(MFFT_EINVAL, "length too large");
        if (d.n == 0) p.empty = true;
        if (d.n > 1) {
            if (mul_overflows(d.n - 1, d.is) || mul_overflows(d.n - 1, d.os))
                return fail(MFFT_EINVAL, "stride * length overflows");
            ext_in += (d.n - 1) * std::llabs(d.is);
            ext_out += (d.n - 1) * std::llabs(d.os);
            if (ext_in > INT64_MAX / 4 || ext_out > INT64_MAX / 4)
                return fail(MFFT_EINVAL, "tensor extent overflows");
        }
        Dim x{d.n, d.is, d.os};
        if (i < rank) N.push_back(x);
        else V.push_back(x);
    }
    if (p.empty) {
        *out = p;
        return MFFT_OK;
    }
    // drop length-1 dims
    N.erase(std::remove_if(N.begin(), N.end(), [](const Dim &d) { return d.n == 1; }), N.end());
    V.erase(std::remove_if(V.begin(), V.end(), [](const Dim &d) { return d.n == 1; }), V.end());
    // any transform dim of length > 2^40 or total > 2^40 elements is refused
    __int128 tot = 1;
    for (const Dim &d : N) tot *= d.n;
    for (const Dim &d : V) tot *= d.n;
    if (tot > ((__int128)1 << 40)) return fail(MFFT_EINVAL, "problem has more than 2^40 elements");

    std::vector<Dim> all = N;
    all.insert(all.end(), V.begin(), V.end());
    if (!outputs_injective(all))
        return fail(MFFT_EINVAL, "two output elements share one address (aliasing output strides)");

    // merge vector loops: a (outer) and b (inner) form one loop when
    // a.is == b.n * b.is and a.os == b.n * b.os
    bool merged = true;
    while (merged && V.size() > 1) {
        merged = false;
        for (size_t i = 0; i < V.size() && !merged; ++i)
            for (size_t j = 0; j < V.size() && !merged; ++j) {
                if (i == j) continue;
                const Dim &a = V[i], &b = V[j];
                if (a.is == b.n * b.is && a.os == b.n * b.os) {
                    Dim m{a.n * b.n, b.is, b.os};
                    V.erase(V.begin() + std::max(i, j));
                    V.erase(V.begin() + std::min(i, j));
                    V.push_back(m);
                    merged = true;
                }
            }
    }
    // order V by input stride, largest first (outer loops first)
    std::sort(V.begin(), V.end(), [](const Dim &a, const Dim &b) {
        if (std::llabs(a.is) != std::llabs(b.is)) return std::llabs(a.is) > std::llabs(b.is);
        return std::llabs(a.os) > std::llabs(b.os);
    });
    p.N = N;
    p.V = V;
    p.n_total = 1;
    for (const Dim &d : N) p.n_total *= d.n;
    p.howmany = 1;
    for (const Dim &d : V) p.howmany *= d.n;
    *out = p;
    return MFFT_OK;
}

int canonicalize_real(int kind, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *hdims, int inplace, int prec, Problem *out)
{
    if (kind != 1 && kind != 2) return fail(MFFT_EINVAL, "unknown real transform kind");
    if (rank < 1 || rank > 8) return fail(MFFT_EINVAL, "real transforms need rank in [1, 8]");
    if (!dims) return fail(MFFT_EINVAL, "dims is NULL");
    // the vector loops alone: validated, merged and ordered as for complex data
    Problem p;
    int rc = canonicalize(0, nullptr, howmany_rank, hdims, inplace, kind == 1 ? -1 : 1, prec, &p);
    if (rc) return rc;
    p.kind = kind;
    std::vector<Dim> N;
    for (int i = 0; i < rank; ++i) {
        const mfft_iodim &d = dims[i];
        if (d.n < 0) return fail(MFFT_EINVAL, "negative length");
        if (d.n > ((int64_t)1 << 40)) return fail(MFFT_EINVAL, "length too large");
        if (d.n == 0) p.empty = true;
        if (mul_overflows(d.n, d.is) || mul_overflows(d.n, d.os))
            return fail(MFFT_EINVAL, "stride * length overflows");
        N.push_back({d.n, d.is, d.os});
    }
    if (p.empty) {
        *out = p;
        return MFFT_OK;
    }
    // outputs: the last dimension holds n/2+1 complex values (forward) or n real
    // values (inverse); the others their full length
    std::vector<Dim> all = p.V;
    __int128 tot = 1;
    for (const Dim &v : p.V) tot *= v.n;
    for (int i = 0; i < rank; ++i) {
        Dim x = N[i];
        if (i == rank - 1 && kind == 1) x.n = x.n / 2 + 1;
        all.push_back(x);
        tot *= x.n;
    }
    if (tot > ((__int128)1 << 40)) return fail(MFFT_EINVAL, "problem has more than 2^40 elements");
    if (!outputs_injective(all))
        return fail(MFFT_EINVAL, "two output elements share one address (aliasing output strides)");
    p.N = N;
    p.n_total = 1;
    for (const Dim &d : N) p.n_total *= d.n;
    *out = p;
    return MFFT_OK;
}

std::string problem_key(const Problem &p)
{
    std::ostringstream s;
    if (p.kind == 1) s << "r2c ";
    else if (p.kind == 2) s << "c2r ";
    s << (p.prec ? "c64" : "c32") << " s" << p.sign << (p.inplace ? " ip" : " op") << " N";
    for (const Dim &d : p.N) s << ":" << d.n << "," << d.is << "," << d.os;
    s << " V";
    for (const Dim &d : p.V) s << ":" << d.n << "," << d.is << "," << d.os;
    return s.str();
}

// ------------------------------------------------------------ number theory

int64_t smallest_prime_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    for (int64_t f = 3; f * f <= n; f += 2)
        if (n % f == 0) return f;
    return n;
}

// Lengths the leaf butterflies factor completely: prime factors 2 .. 13.
bool is_smooth(int64_t n)
{
    if (n < 1) return false;
    for (int64_t f : {2, 3, 5, 7, 11, 13})
        while (n % f == 0) n /= f;
    return n == 1;
}

// Lengths the leaves with 24 elements per thread also factor: prime factors
// up to 23 (radices 17, 19, 23 besides those of is_smooth).
bool is_smooth23(int64_t n)
{
    if (n < 1) return false;
    for (int64_t f : {2, 3, 5, 7, 11, 13, 17, 19, 23})
        while (n % f == 0) n /= f;
    return n == 1;
}

static int64_t powmod(int64_t b, int64_t e, int64_t m)
{
    int64_t r = 1 % m;
    b %= m;
    while (e > 0) {
        if (e & 1) r = (int64_t)((__int128)r * b % m);
        b = (int64_t)((__int128)b * b % m);
        e >>= 1;
    }
    return r;
}

// Smallest generator of the multiplicative group mod prime p.
int64_t primitive_root(int64_t p)
{
    if (p == 2) return 1;
    std::vector<int64_t> fac;
    int64_t m = p - 1;
    for (int64_t f = 2; f * f <= m; ++f)
        if (m % f == 0) {
            fac.push_back(f);
            while (m % f == 0) m /= f;
        }
    if (m > 1) fac.push_back(m);
    for (int64_t g = 2; g < p; ++g) {
        bool ok = true;
        for (int64_t f : fac)
            if (powmod(g, (p - 1) / f, p) == 1) {
                ok = false;
                break;
            }
        if (ok) return g;
    }
    return 0;
}

// Division by an invariant d via multiply-high (round-up method):
// q = (umulhi(b, magic) + b) >> shift, exact for b < 2^24 and d < 2^24.
void div_magic(uint32_t d, uint32_t *magic, int *shift)
{
    int l = 0;
    while (((uint64_t)1 << l) < d) ++l;
    const uint64_t m = (((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1;
    *magic = (uint32_t)m;
    *shift = l;
}

}  // namespace mfft

extern "C" int mfft_problem_check(int rank, const mfft_iodim *dims, int howmany_rank,
                                  const mfft_iodim *howmany_dims, int inplace, int sign,
                                  mfft_prec prec)
{
    mfft::Problem p;
    return mfft::canonicalize(rank, dims, howmany_rank, howmany_dims, inplace, sign, (int)prec, &p);
}

extern "C" int mfft_problem_check_real(int inverse, int rank, const mfft_iodim *dims,
                                       int howmany_rank, const mfft_iodim *howmany_dims,
                                       int inplace, mfft_prec prec)
{
    if (inverse != 0 && inverse != 1) return mfft::fail(MFFT_EINVAL, "inverse must be 0 or 1");
    mfft::Problem p;
    return mfft::canonicalize_real(inverse ? 2 : 1, rank, dims, howmany_rank, howmany_dims, inplace,
                                   (int)prec, &p);
}
