/*
 * mfft: complex DFTs over I/O tensors on AMD Instinct MI355X (gfx950).
 *
 * The problem statement is the one of Johnson & Frigo, "Implementing FFTs in
 * Practice", Section 4.1 ("The problem to be solved"): a DFT problem
 * dft(N, V, I, O) is a rank-r transform size N and a vector size V, both
 * I/O tensors -- sets of I/O dimensions (n, is, os) with a non-negative length n
 * and integer input/output strides -- plus an input pointer I and an output
 * pointer O.  Every I/O dimension of V is a loop of independent transforms,
 * every I/O dimension of N one dimension of the (separable) transform.  I = O
 * is the in-place case.
 *
 * Conventions fixed by this library where the paper leaves a choice:
 *   - strides count complex elements of the plan's precision; data is
 *     interleaved (re, im);
 *   - sign -1 is the forward DFT of eq. (dft), Section 2,
 *     Y[k] = sum_l X[l] exp(-2 pi i l k / n); sign +1 conjugates the exponent;
 *     neither direction is normalized (forward then inverse = n * identity);
 *   - a problem with any n = 0 is a valid no-op; rank 0 is a copy;
 *   - the input is read as it was before the call, also when I = O with
 *     different input and output strides (scratch memory is used then);
 *   - two different (vector, frequency) indices writing one output address is
 *     an error (MFFT_EINVAL).
 *
 * All functions return a status code (0 = success, < 0 = error) and never
 * throw; mfft_last_error() holds a thread-local message for the last failure.
 * Device pointers are plain HIP device addresses; streams are hipStream_t
 * passed as void* (NULL = the default stream).
 */
#ifndef MFFT_H
#define MFFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define MFFT_OK        0
#define MFFT_EINVAL   (-1)  /* malformed problem or argument                    */
#define MFFT_ENOTSUP  (-2)  /* well-formed problem this build cannot plan       */
#define MFFT_ENOMEM   (-3)  /* device or host allocation failed                 */
#define MFFT_EHIP     (-4)  /* a HIP runtime call failed (text in last_error)   */
#define MFFT_EALIGN   (-5)  /* execute pointers contradict what the plan assumed */
#define MFFT_EBUDGET  (-6)  /* request can never fit the server's HBM budget    */
#define MFFT_ESTATE   (-7)  /* object in the wrong state (stopped, unknown id)  */
#define MFFT_ETIMEOUT (-8)  /* wait expired before completion                   */
#define MFFT_ECANCELED (-9) /* request was cancelled                            */
#define MFFT_ENOWISDOM (-10) /* MFFT_WISDOM_ONLY and no stored plan matches      */

/* ------------------------------------------------------------------ problem */
/* One I/O dimension (Section 4.1): length n >= 0, input stride is, output
 * stride os, both in complex elements, either sign. */
typedef struct {
    int64_t n, is, os;
} mfft_iodim;

/* Precision of data and arithmetic: interleaved single or double complex. */
typedef enum { MFFT_C32 = 0, MFFT_C64 = 1 } mfft_prec;

/* Planner rigor (Section 4.3, "The FFTW planner"). */
#define MFFT_ESTIMATE    0u  /* heuristic cost model, no timing                 */
#define MFFT_MEASURE     1u  /* time candidate plans on the stream, keep fastest */
#define MFFT_WISDOM_ONLY 2u  /* only a stored plan; else MFFT_ENOWISDOM          */
#define MFFT_NO_WISDOM   4u  /* neither consult nor record stored plans          */
/* Accuracy ablation of Section 6 (FP32 plans only, not for production use):
 * the stage twiddle tables are evaluated in FP32 arithmetic (angle, sine and
 * cosine) instead of FP64 rounded once to FP32.  The index product is still
 * reduced exactly in integer arithmetic. */
#define MFFT_FP32_TWIDDLES 8u
/* In-place plans that need no scratch memory (Section 4.2's in-place plans):
 * a transform along a dimension too long for one pass, n = q*q or n = 2*q*q
 * with q (and 2q) one pass, runs as columns (with the Cooley-Tukey twiddle),
 * rows, an in-place q x q transpose (of both halves for 2*q*q) and, for
 * 2*q*q, an in-place interleave of the halves' rows, all in the caller's
 * buffer, instead of two passes through a scratch copy (one or two more
 * passes over HBM, no scratch).  Planning fails with MFFT_ENOTSUP when the
 * problem has no such plan (a multi-pass length of another form, prime sizes
 * that need a convolution buffer, in-place
 * problems whose input and output strides differ, and real-data transforms
 * that need a packed copy).  Applies to in-place problems; out-of-place plans
 * use no scratch anyway except for prime and real-data cases, which then also
 * fail with MFFT_ENOTSUP. */
#define MFFT_NO_SCRATCH 16u

/* Optional device allocator (e.g. a framework's caching allocator).  alloc
 * returns NULL on failure.  NULL allocator = hipMalloc / hipFree. */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *ctx);
    void (*free)(void *ptr, void *stream, void *ctx);
    void *ctx;
} mfft_allocator;

typedef struct mfft_plan_s *mfft_plan;

/* Description of a plan (for reports and tests). */
typedef struct {
    int prec;                 /* mfft_prec                                     */
    int sign;                 /* -1 or +1                                      */
    int rank, howmany_rank;   /* after canonicalization                        */
    int inplace;              /* plan expects in == out                        */
    int n_passes;             /* kernel launches per execute                   */
    int64_t n_total;          /* product of transform lengths (real plans: n)  */
    int64_t howmany;          /* product of vector lengths                     */
    double flops;             /* nominal 5 N log2 N per transform (real plans:
                               * 2.5 N log2 N), x howmany                     */
    double bytes_compulsory;  /* read input once + write output once           */
    double bytes_passes;      /* bytes the passes move to and from HBM         */
    size_t scratch_bytes;     /* device scratch owned by the plan              */
    size_t table_bytes;       /* device twiddle / chirp / index tables         */
    char desc[1024];          /* human-readable pass list                      */
    /* The radices each pass executes (its Stockham stages in order, Section 2;
     * one transform of the product per line), the passes in launch order and
     * each list closed by a 0; a pass that transforms nothing (a copy, a
     * transpose, a real-data step) contributes the 0 alone.  At most
     * MFFT_INFO_RADICES entries; n_radices counts those filled (a longer list
     * is cut there). */
#define MFFT_INFO_RADICES 64
    int n_radices;
    int radices[MFFT_INFO_RADICES];
} mfft_plan_info_t;

/*
 * Validate a problem without touching the GPU (host-only).
 *   rank, dims:                 transform size N (rank <= 8); dims may be NULL
 *                               when rank == 0.
 *   howmany_rank, howmany_dims: vector size V (rank <= 8).
 *   inplace:                    1 if the caller will pass in == out.
 *   sign:                       -1 or +1.   prec: MFFT_C32 or MFFT_C64.
 * Returns MFFT_OK, MFFT_EINVAL (bad lengths, strides that overflow, outputs
 * that alias, bad sign/prec) or MFFT_ENOTSUP.
 */
int mfft_problem_check(int rank, const mfft_iodim *dims, int howmany_rank,
                       const mfft_iodim *howmany_dims, int inplace, int sign, mfft_prec prec);

/*
 * Plan dft(N, V, I, O) (Section 4: a plan is a composition of algorithmic
 * steps chosen by the planner; here each step is one GPU pass).
 * Arguments as for mfft_problem_check, plus
 *   flags:      MFFT_ESTIMATE / MFFT_MEASURE / MFFT_WISDOM_ONLY | MFFT_NO_WISDOM
 *               (| MFFT_FP32_TWIDDLES for the accuracy ablation,
 *               | MFFT_NO_SCRATCH for plans without scratch); other bits,
 *               or MFFT_FP32_TWIDDLES with MFFT_C64, give EINVAL before any
 *               device work;
 *   alloc:      allocator for the plan's tables and scratch (NULL = hipMalloc);
 *   hip_stream: stream for table generation and measurement.
 * On success *out receives a plan that owns its device tables and scratch.
 * Table generation is enqueued on hip_stream; executing on another stream
 * requires the caller to order the two streams.  Planning is serialized by an
 * internal lock.  Errors: EINVAL, ENOTSUP, ENOMEM, EHIP, ENOWISDOM.
 */
int mfft_plan_dft(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                  const mfft_iodim *howmany_dims, int inplace, int sign, mfft_prec prec,
                  unsigned flags, const mfft_allocator *alloc, void *hip_stream);

/*
 * Real-data transforms.  A DFT of real input is conjugate symmetric,
 * Y[n-k] = conj(Y[k]), so outputs 0 .. n/2 determine it (the real-data case
 * Sections 5 and 7 single out: about half the work).  rank 1 .. 8; the LAST
 * dimension, dims[rank-1] with n real points, is the one halved (n/2+1
 * complex values); the other dimensions keep their length.  Below, "the
 * dimension" is dims[rank-1]; the other dims and the howmany dims take strides
 * in the same units as it on each side.
 *   mfft_plan_dft_r2c: forward (sign -1) DFT of real inputs (input strides
 *     in real elements of the precision) to complex outputs (output strides in
 *     complex elements).
 *   mfft_plan_dft_c2r: the unnormalized inverse (sign +1) from the half
 *     spectrum (input strides in complex elements; along the halved dimension
 *     the imaginary parts of bins 0 and n/2, zero for a conjugate-symmetric
 *     spectrum, are ignored; for rank > 1 the input must be such a spectrum)
 *     to real outputs (output strides in real elements).
 * c2r(r2c(x)) = N x (N = product of the lengths).  inplace = 1: input and
 * output share one buffer (the plan
 * reads the input completely before writing).  Real buffers must be aligned
 * to the complex element size like complex ones.  Even n with unit real
 * stride and even real vector strides runs a complex DFT of length n/2 plus
 * one elementwise pass; other shapes run a length-n complex DFT.  Executed
 * with mfft_execute / mfft_execute_scratch; other arguments and errors as for
 * mfft_plan_dft (MFFT_FP32_TWIDDLES included).
 */
/* Host-only validation of a real-data problem (inverse 0: r2c, 1: c2r);
 * returns what planning would for the problem itself (MFFT_OK, MFFT_EINVAL,
 * MFFT_ENOTSUP), without touching the GPU. */
int mfft_problem_check_real(int inverse, int rank, const mfft_iodim *dims, int howmany_rank,
                            const mfft_iodim *howmany_dims, int inplace, mfft_prec prec);
int mfft_plan_dft_r2c(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *howmany_dims, int inplace, mfft_prec prec, unsigned flags,
                      const mfft_allocator *alloc, void *hip_stream);
int mfft_plan_dft_c2r(mfft_plan *out, int rank, const mfft_iodim *dims, int howmany_rank,
                      const mfft_iodim *howmany_dims, int inplace, mfft_prec prec, unsigned flags,
                      const mfft_allocator *alloc, void *hip_stream);

/*
 * Enqueue the transform on hip_stream (asynchronous; no allocation, no
 * synchronization, so it can be captured in a HIP graph).  `in` and `out` point
 * at element (0,...,0) of the input and output tensors.  An out-of-place plan
 * (inplace = 0) never writes the input; in == out is rejected with
 * MFFT_EALIGN for it, as is in != out for an in-place plan or a pointer not
 * aligned to the complex element size.  Calls on one plan must not overlap
 * in time (they share the plan's scratch); use mfft_execute_scratch with
 * distinct scratch buffers for concurrent executions.
 */
int mfft_execute(mfft_plan plan, const void *in, void *out, void *hip_stream);

/* As mfft_execute, with caller-owned scratch of at least info.scratch_bytes
 * (NULL allowed when that size is 0). */
int mfft_execute_scratch(mfft_plan plan, const void *in, void *out, void *scratch,
                         void *hip_stream);

/*
 * For callers that cannot allocate device memory at execution time (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): as
 * mfft_execute_scratch, with the scratch taken from a fixed array of
 * MFFT_STATIC_SCRATCH_BYTES that the library reserves on each GPU it runs on
 * (held until the process ends).  The call allocates and frees nothing.
 * The plan's device must be current.  A plan whose info.scratch_bytes exceeds
 * MFFT_STATIC_SCRATCH_BYTES is refused with MFFT_ENOMEM before any launch;
 * a plan without scratch runs as with mfft_execute.  Every call on one GPU
 * shares that GPU's array, and the array keeps the last call's contents (no
 * plan reads scratch it has not written in the same call): calls that overlap
 * in time on one GPU, on any streams, race and must be ordered by the caller.
 * Other arguments and errors as for mfft_execute.
 */
#define MFFT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mfft_execute_static_scratch(mfft_plan plan, const void *in, void *out, void *hip_stream);

/* Fill *info for a plan. */
int mfft_plan_info(mfft_plan plan, mfft_plan_info_t *info);

/* Free the plan's device memory (stream-ordered on the plan's stream). */
int mfft_plan_destroy(mfft_plan plan);

/* ------------------------------------------------------------------ batch */
/*
 * Many planned transforms executed as one workload (the vector-loop rule of
 * Section 4.2 extended across plans): pass k of every plan runs in one
 * launch per kernel family, one workgroup per tile of a list ordered largest
 * line first, so uneven sizes balance across the GPU; passes of the
 * specialized power-of-two leaf kernel run in one launch per length and tile
 * kind, with the same results as the plans alone.  The launches of one pass
 * index are independent and run on up to four concurrent lanes (the caller's
 * stream and three of the batch's own, forked from and joined back to it;
 * parallel branches of the graph).  Column passes move 128-byte runs: items
 * whose data start on a 128-byte boundary run them about twice as fast as
 * misaligned ones.
 *   count, plans, ins, outs: plan i runs on ins[i] -> outs[i] (device
 *       pointers with the plan's in-place rule); plans must outlive the batch;
 *       a plan that owns scratch may appear at most once.
 *   flags: MFFT_BATCH_GRAPH captures the launches in a HIP graph at creation;
 *       execute then launches the graph.
 * Execution is asynchronous on hip_stream and allocates nothing; executions
 * of one batch must not overlap (they share its lanes).  Errors: EINVAL (bad
 * arguments, shared scratch), ENOMEM, EHIP.
 */
typedef struct mfft_batch_s *mfft_batch;
#define MFFT_BATCH_GRAPH 1u

int mfft_batch_create(mfft_batch *out, int count, const mfft_plan *plans, const void *const *ins,
                      void *const *outs, unsigned flags, void *hip_stream);
int mfft_batch_execute(mfft_batch batch, void *hip_stream);
/* Number of kernel launches per execute and total tiles. */
int mfft_batch_info(mfft_batch batch, int *launches, int64_t *tiles);
int mfft_batch_destroy(mfft_batch batch);

/* ------------------------------------------------------------------ server */
/*
 * Request server with continuous batching.  Requests (any problem the planner
 * accepts) are queued; a scheduler thread admits them in arrival order while
 * their memory fits the HBM budget and fewer than max_inflight are on the GPU,
 * and launches everything admitted since the last launch as one batch (see
 * mfft_batch_*) on the next of n_streams streams, so requests that arrive while
 * others run are admitted as memory frees and overlap on the device.  Plans and
 * their twiddle tables stay resident in a cache keyed by the problem; a
 * request whose plan is not cached is planned by a separate planner thread
 * while the scheduler keeps admitting and retiring requests whose plans exist
 * (admission is in arrival order among requests whose plan is ready; the
 * first of them that does not fit the memory left blocks the others).
 *
 *   hbm_budget_bytes: device memory the server may hold: request outputs and
 *       scratch, launch descriptors and the cached plans' tables (the budget
 *       is reserved once at creation; cached plans no request uses are evicted,
 *       least recently used first, when memory is short).  Transient buffers of
 *       planning itself (the FP64 sub-transforms that build prime-size tables)
 *       come from hipMalloc and are freed before planning returns.
 *   max_inflight: admitted-but-unfinished request limit (>= 1); n_streams >= 1.
 *   alloc: allocator for the budget's one reservation (NULL = hipMalloc);
 *       called once at creation and once (free) at destruction.
 * A request's input must stay valid until it completes.  If in_stream is not
 * NULL, the request runs after the work enqueued on that stream before the
 * submission (an event is recorded on it at submission); with NULL the input
 * must be complete when submitted.  If out is NULL the server allocates the
 * output inside the budget; read it with mfft_server_output and give it back
 * with mfft_server_release.
 */
typedef struct mfft_server_s *mfft_server;

typedef struct {
    int rank;
    mfft_iodim dims[8];
    int howmany_rank;
    mfft_iodim howmany_dims[8];
    int sign;            /* -1 or +1 */
    mfft_prec prec;
    const void *in;      /* device input tensor, element (0,...,0)              */
    void *out;           /* device output, or NULL = allocate in the budget      */
    double arrival;      /* steady-clock seconds of arrival (0 = at submission)  */
    void *in_stream;     /* stream producing the input (hipStream_t), or NULL    */
} mfft_request;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, failed, cancelled;
    uint64_t launches;       /* batched launches (ticks)                           */
    double p50_ms, p99_ms;   /* arrival -> completion observed, completed requests */
    double mean_ms, max_ms;
    double busy_s;           /* time with at least one launch on the GPU           */
    double flops;            /* nominal 5 N log2 N flops of completed requests     */
    double bytes;            /* compulsory bytes of completed requests             */
    size_t bytes_in_use, peak_bytes;   /* within the budget                        */
    size_t plan_bytes;       /* resident plan tables (inside the budget, counted
                              * in bytes_in_use and peak_bytes)                  */
    int plans_cached;
    int max_inflight_seen;
    int plans_evicted;       /* cached plans dropped to make room                  */
} mfft_server_stats_t;

/* Request status reported by mfft_server_wait. */
#define MFFT_REQ_PENDING  1
#define MFFT_REQ_RUNNING  2
#define MFFT_REQ_DONE     0

int mfft_server_create(mfft_server *out, size_t hbm_budget_bytes, int max_inflight, int n_streams,
                       const mfft_allocator *alloc);
/* EINVAL/ENOTSUP for a bad problem, EBUDGET if it can never fit the budget. */
int mfft_server_submit(mfft_server server, const mfft_request *req, uint64_t *ticket);
/* Wait up to timeout_ms (< 0: forever).  *status: MFFT_REQ_DONE, a negative
 * error code of the request, or MFFT_REQ_PENDING / RUNNING on timeout
 * (then the call returns MFFT_ETIMEOUT). */
int mfft_server_wait(mfft_server server, uint64_t ticket, int timeout_ms, int *status);
int mfft_server_output(mfft_server server, uint64_t ticket, void **out);
/* Forget a finished request and free its server-allocated output. */
int mfft_server_release(mfft_server server, uint64_t ticket);
/* Cancel a request that has not been admitted (ESTATE if already running). */
int mfft_server_cancel(mfft_server server, uint64_t ticket);
int mfft_server_stats(mfft_server server, mfft_server_stats_t *stats);
/* Clear the counters and latency samples (e.g. after a warm-up phase). */
int mfft_server_reset_stats(mfft_server server);
/* Stop accepting, cancel requests not yet admitted (their wait returns
 * MFFT_ECANCELED), finish in-flight work, free everything. */
int mfft_server_destroy(mfft_server server);

/* ------------------------------------------------------------------ wisdom */
/* Stored plans (Section 4.3: plans can be precomputed and loaded later).  The
 * text records, per canonical problem, precision, device architecture and
 * library version, the choices the planner made.  export allocates *buf with
 * malloc-compatible memory released by mfft_free. */
int mfft_wisdom_export(char **buf, size_t *len);
int mfft_wisdom_import(const char *buf, size_t len);
int mfft_wisdom_forget(void);
void mfft_free(void *p);

/* ------------------------------------------------------------------ misc */
/* Thread-local text of the last error on this thread ("" if none). */
const char *mfft_last_error(void);
/* Library version string. */
const char *mfft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MFFT_H */
