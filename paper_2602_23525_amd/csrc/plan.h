// Host-side plan structures: canonical problems, passes, plans.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/mfft.h"
#include "internal.h"
#include "kernels.h"

namespace mfft {

struct Dim {
    int64_t n, is, os;
};

// dft(N, V, I, O) after canonicalization (Section 4.1): no length-1
// dimensions, mergeable vector loops merged.
struct Problem {
    std::vector<Dim> N, V;
    // 0: complex dft(N, V, I, O); 1: real input, half spectrum out (N has one
    // dim: n real points, is in real / os in complex elements); 2: the inverse
    // (is in complex / os in real elements).  V strides use the same units.
    int kind = 0;
    int sign = -1;
    int prec = 0;          // 0 = C32, 1 = C64
    bool inplace = false;
    bool empty = false;    // some length was 0: nothing to do
    int64_t n_total = 1, howmany = 1;
};

// Status + message helpers (thread-local error text).
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// Validate and canonicalize; returns MFFT_OK or an error code (message set).
int canonicalize(int rank, const mfft_iodim *dims, int howmany_rank, const mfft_iodim *hdims,
                 int inplace, int sign, int prec, Problem *out);
// The same for real-data problems (kind 1 or 2).
int canonicalize_real(int kind, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *hdims, int inplace, int prec, Problem *out);
std::string problem_key(const Problem &p);

// Buffer ids a pass reads and writes.
enum : int { BUF_IN = 0, BUF_OUT = 1, BUF_SCRATCH = 2 };

struct Pass {
    int kind = 0;            // 0 = FFT tile pass, 1 = rank-0 copy, 2 = real-data step,
                             // 3 = in-place square transpose, 4 = in-place item permutation
    PassArgs a{};            // pointers filled at execute time (except tables)
    CopyArgs c{};
    RealArgs r{};
    TransposeArgs t{};
    PermuteArgs pm{};
    int src = BUF_IN, dst = BUF_OUT;
    int64_t src_off = 0, dst_off = 0;       // complex elements (scratch: region offset)
    int64_t aux_off = -1;                    // bytes into scratch for Rader aux, or -1
    int emax = 16;
    int kernel = 0;          // 0 = generic tile kernel, 1 = specialized leaf kernel
    int variant = 0;         // leaf kernel variant bits
    int persistent = 0;      // leaf kernel: grid of resident workgroups instead of one per tile
    int64_t grid = 0;        // leaf kernel grid (workgroups)
    int prec = 0;
    size_t lds_bytes = 0;
    double bytes = 0;        // HBM bytes the pass moves (algorithmic)
    std::string desc;
};

// Tunable choice of the specialized leaf kernel (what measure mode times and
// wisdom records): variant bits (see k_leaf.hip) and grid kind.
struct LeafTune {
    int variant = 0;
    int persistent = 0;
};

// Structural choices for the lines of one length (what measure mode times and
// wisdom stores besides kernel variants; zero / empty = the estimate's).
struct StructChoice {
    std::vector<int> rad;   // radix sequence of a generic-kernel leaf of this length
    int bt = 0;             // lines per row tile of that leaf
    int64_t split = 0;      // two-pass Cooley-Tukey: length of the first pass's lines
    int prime = 0;          // prime length: 1 Rader, 2 Bluestein
    int64_t M = 0;          // Bluestein's convolution length
    int emax = 0;           // elements per thread of a generic leaf (16 or 24)
    bool empty() const { return rad.empty() && !bt && !split && !prime && !M && !emax; }
};

struct DeviceAlloc {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct PlanImpl {
    Problem prob;
    unsigned flags = 0;
    std::vector<Pass> passes;
    std::vector<DeviceAlloc> tables;
    size_t table_bytes = 0;
    size_t scratch_bytes = 0;
    void *scratch = nullptr;             // plan-owned scratch (may be null)
    mfft_allocator alloc{};
    bool has_alloc = false;
    hipStream_t stream = nullptr;
    std::string desc;
    double bytes_passes = 0;
    int device = 0;
    bool from_wisdom = false;
    std::map<int64_t, StructChoice> overrides;   // by line length
};

}  // namespace mfft

struct mfft_plan_s {
    mfft::PlanImpl impl;
};

namespace mfft {

// Device memory through the plan's allocator.
void *dev_alloc(PlanImpl *p, size_t bytes);
void dev_free(PlanImpl *p, void *ptr, size_t bytes);

// Build the pass list and tables of a plan (Section 4.2 plan steps).
int build_plan(PlanImpl *p);
LeafTune leaf_default(int prec, int n, double in_bytes);
void apply_leaf_tune(Pass *ps, const LeafTune &t);

// Planner rigor (Section 4.3): time the candidate kernel variants of every
// tunable pass on the plan's stream and keep the fastest; apply / record wisdom.
int measure_plan(PlanImpl *p);
std::string plan_choices(const PlanImpl *p);
bool apply_choices(PlanImpl *p, const std::string &text);
// Structural choices: the candidates for lines of length n (the estimate's
// own first), measuring them (rebuilding the plan per candidate), and their
// text form in wisdom ("n=1000:r=10.10.10:b=5", ...).
std::vector<StructChoice> structure_candidates(const PlanImpl *p, int64_t n);
int measure_structure(PlanImpl *p);
std::string choice_text(int64_t n, const StructChoice &c);
bool parse_choice(const std::string &text, int64_t *n, StructChoice *c);
bool parse_structure(const std::string &text, std::map<int64_t, StructChoice> *out);
// Free the plan's tables and passes and build it again (with p->overrides).
int rebuild_plan(PlanImpl *p);

// Enqueue the passes.
int run_plan(const PlanImpl *p, const void *in, void *out, void *scratch, hipStream_t s);

// A pass with its buffer pointers resolved for given in/out/scratch pointers.
PassArgs resolve_pass(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch);
CopyArgs resolve_copy(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch);
RealArgs resolve_real(const PlanImpl *p, const Pass &ps, const void *in, void *out, void *scratch);
TransposeArgs resolve_transpose(const PlanImpl *p, const Pass &ps, const void *in, void *out,
                                void *scratch);
PermuteArgs resolve_permute(const PlanImpl *p, const Pass &ps, const void *in, void *out,
                            void *scratch);
// Lines per tile of a generic-kernel row tile (see plan.cpp).
int row_lines_per_tile(int n, int tpt, int prec, int64_t lines, int emax = 0);
// LDS layouts of the generic kernel's stage boundaries (StageDesc rd_stride,
// rd_shift, wr_shift) for a leaf of nst stages st[0..nst) with R, Ns, nb set.
void lds_layouts(int n, int nst, int tpt, int lds_stride, int emax, int eb, StageDesc *st);
// LDS bytes the generic tile kernel needs for a pass.
size_t generic_lds_bytes(const Pass &ps);

// Wisdom store (text): key -> choice string.
bool wisdom_lookup(const std::string &key, std::string *val);
void wisdom_record(const std::string &key, const std::string &val);

// Internal planner flag (never accepted from the C ABI): the plan allocates no
// scratch of its own; its executions take scratch from the caller (the
// request server allocates it per request inside its budget).
constexpr unsigned kPlanNoOwnScratch = 1u << 30;

// Plan under the global planner lock, with internal flags allowed.
int plan_dft_locked(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                    const mfft_iodim *hdims, int inplace, int sign, int prec, unsigned flags,
                    const mfft_allocator *alloc, hipStream_t stream);

// Plan without taking the global planner lock (FP64 sub-plans for tables).
int plan_internal(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                  const mfft_iodim *hdims, int inplace, int sign, int prec, hipStream_t stream,
                  unsigned flags = 0, const mfft_allocator *alloc = nullptr, int kind = 0);

int64_t smallest_prime_factor(int64_t n);
bool is_smooth(int64_t n);
bool is_smooth23(int64_t n);
int64_t primitive_root(int64_t p);
void div_magic(uint32_t d, uint32_t *magic, int *shift);

}  // namespace mfft
