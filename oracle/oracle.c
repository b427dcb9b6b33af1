/*
 * FP64 CPU oracle for the complex DFT over I/O tensors.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls, links or loads this
 * file; only the tests, the smoke check and the benchmark's CPU-baseline leg use
 * it.  It shares no code, header, table or constant with the GPU library.
 *
 * What it computes (Johnson & Frigo, "Implementing FFTs in Practice"):
 *   * the forward DFT of eq. (dft), Section 2: Y[k] = sum_l X[l] w^(l k),
 *     w = exp(sign * 2 pi i / n); sign = -1 is the paper's forward transform,
 *     sign = +1 the conjugate-exponent transform, both unnormalized;
 *   * over an I/O tensor problem dft(N, V, I, O) of Section 4.1: every vector
 *     loop of V indexes an independent transform, every I/O dimension of N is
 *     one dimension of a separable multi-dimensional DFT (same sign in every
 *     dimension), strides counted in complex elements;
 *   * the input is read from a snapshot taken before anything is written, which
 *     fixes the meaning of in-place and overlapping problems.
 *
 * Algorithms (each a plain statement of the paper's definitions):
 *   O1 direct:    eq. (dft) summed in long double; w^m taken from a table indexed
 *                 by (l*k mod n), reduced in 64-bit integers.
 *   O2 recursive: eq. (ct) with the radix n2 = p, the smallest prime factor of n
 *                 (decimation in time, Section 2); Algorithm 1 is the p = 2 case.
 *                 Out-of-place, in-order output, no separate digit reversal.
 *                 Prime lengths fall back to O1.
 *   O3 Bluestein: the chirp-z identity l*k = (l^2 + k^2 - (k-l)^2)/2 turns the
 *                 DFT into a linear convolution (Section 4.2, "Plans for prime
 *                 sizes"), evaluated with O2 at a power-of-two length >= 2n-1.
 *   MD direct:    the multi-dimensional definition summed directly (tiny shapes).
 *
 * Twiddle values: exp(2 pi i m / n) is evaluated in long double on an angle
 * reduced to the first octant with integer arithmetic, so that the eighth roots
 * of unity are exact and w^(n-m) is exactly conj(w^m) (Section 6 asks for
 * twiddles accurate to machine precision).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double ld;

typedef struct { int64_t n, is, os; } oracle_iodim;

enum { OR_AUTO = 0, OR_DIRECT = 1, OR_RECURSIVE = 2, OR_BLUESTEIN = 3, OR_MD_DIRECT = 4 };

/* ---------------------------------------------------------------- roots */

/* (c, s) = (cos, sin)(2 pi m / n) for 0 <= m < n, octant-reduced. */
static void unit_root(int64_t m, int64_t n, ld *c, ld *s)
{
    m %= n;
    if (m < 0) m += n;
    /* 2 pi m / n = (pi/4) * (8m / n); split 8m = oct * n + r with 0 <= r < n. */
    __int128 t = (__int128)8 * m;
    int oct = (int)(t / n);
    int64_t r = (int64_t)(t - (__int128)oct * n);
    if (oct & 1) r = n - r;                      /* measure from the far edge */
    ld th = (3.14159265358979323846264338327950288L / 4.0L) * ((ld)r / (ld)n);
    ld a = cosl(th), b = sinl(th);
    switch (oct) {
    case 0: *c = a;  *s = b;  break;            /* th            */
    case 1: *c = b;  *s = a;  break;            /* pi/2 - th     */
    case 2: *c = -b; *s = a;  break;            /* pi/2 + th     */
    case 3: *c = -a; *s = b;  break;            /* pi - th       */
    case 4: *c = -a; *s = -b; break;            /* pi + th       */
    case 5: *c = -b; *s = -a; break;            /* 3pi/2 - th    */
    case 6: *c = b;  *s = -a; break;            /* 3pi/2 + th    */
    default: *c = a; *s = -b; break;            /* 2pi - th      */
    }
}

/* Table W[m] = exp(sign * 2 pi i m / n), m < n, stored as long double pairs. */
static ld *root_table(int64_t n, int sign)
{
    ld *w = (ld *)malloc(sizeof(ld) * 2 * (size_t)(n > 0 ? n : 1));
    if (!w) return NULL;
    for (int64_t m = 0; m < n; ++m) {
        ld c, s;
        unit_root(m, n, &c, &s);
        w[2 * m] = c;
        w[2 * m + 1] = sign < 0 ? -s : s;
    }
    return w;
}

void oracle_root(int64_t m, int64_t n, int sign, double *out2)
{
    ld c, s;
    unit_root(m, n, &c, &s);
    out2[0] = (double)c;
    out2[1] = (double)(sign < 0 ? -s : s);
}

/* ---------------------------------------------------------------- O1 */

/* Y[k*ys] = sum_l X[l*xs] W[(l*k) mod n] with a precomputed table W (size n). */
static void direct_1d(int64_t n, const ld *W, const double *x, int64_t xs, double *y, int64_t ys)
{
    for (int64_t k = 0; k < n; ++k) {
        ld re = 0.0L, im = 0.0L;
        int64_t idx = 0;                          /* (l*k) mod n, kept reduced */
        for (int64_t l = 0; l < n; ++l) {
            ld xr = x[2 * l * xs], xi = x[2 * l * xs + 1];
            ld wr = W[2 * idx], wi = W[2 * idx + 1];
            re += xr * wr - xi * wi;
            im += xr * wi + xi * wr;
            idx += k;
            if (idx >= n) idx -= n;
        }
        y[2 * k * ys] = (double)re;
        y[2 * k * ys + 1] = (double)im;
    }
}

void oracle_dft_direct_1d(int64_t n, int sign, const double *x, int64_t xs, double *y, int64_t ys)
{
    if (n <= 0) return;
    ld *W = root_table(n, sign);
    direct_1d(n, W, x, xs, y, ys);
    free(W);
}

/* ---------------------------------------------------------------- O2 */

static int64_t smallest_factor(int64_t n)
{
    if (n % 2 == 0) return 2;
    for (int64_t f = 3; f * f <= n; f += 2)
        if (n % f == 0) return f;
    return n;
}

/*
 * y[0..n) = DFT of x[l * xs], l < n, using the root table Wtop of length ntop,
 * where n divides ntop: w_n^e = Wtop[e * (ntop / n)].
 * Decimation in time with radix p (eq. ct with n1 = m = n/p, n2 = p):
 *   Z_j = DFT_m of x[(l1 p + j) xs]               (inner sums, recursion)
 *   Y[k1 + k2 m] = sum_j (w_n^(j k1) Z_j[k1]) w_p^(j k2)   (twiddle, outer sums)
 */
static void rec_1d(int64_t n, const double *x, int64_t xs, double *y,
                   const ld *Wtop, int64_t ntop, double *work)
{
    if (n == 1) {
        y[0] = x[0];
        y[1] = x[1];
        return;
    }
    int64_t p = smallest_factor(n);
    int64_t step = ntop / n;                      /* w_n^e = Wtop[e*step] */
    if (p == n) {                                 /* prime length: definition */
        for (int64_t k = 0; k < n; ++k) {
            ld re = 0.0L, im = 0.0L;
            int64_t idx = 0;
            for (int64_t l = 0; l < n; ++l) {
                ld xr = x[2 * l * xs], xi = x[2 * l * xs + 1];
                const ld *w = Wtop + 2 * (idx * step);
                re += xr * w[0] - xi * w[1];
                im += xr * w[1] + xi * w[0];
                idx += k;
                if (idx >= n) idx -= n;
            }
            y[2 * k] = (double)re;
            y[2 * k + 1] = (double)im;
        }
        return;
    }
    int64_t m = n / p;
    /* inner DFTs: Z_j stored at work[j*m .. j*m+m) */
    for (int64_t j = 0; j < p; ++j)
        rec_1d(m, x + 2 * j * xs, p * xs, work + 2 * j * m, Wtop, ntop, y);
    /* twiddle + outer size-p DFTs */
    for (int64_t k1 = 0; k1 < m; ++k1) {
        for (int64_t k2 = 0; k2 < p; ++k2) {
            ld re = 0.0L, im = 0.0L;
            for (int64_t j = 0; j < p; ++j) {
                /* exponent of w_n: j*k1 + j*k2*m  (= j * (k1 + k2 m)), mod n;
                 * j < p <= n and k1 + k2 m < n, so the product fits in 64 bits
                 * for every n below 2^31 */
                int64_t e = (j * (k1 + k2 * m)) % n;
                const ld *w = Wtop + 2 * (e * step);
                ld zr = work[2 * (j * m + k1)], zi = work[2 * (j * m + k1) + 1];
                re += zr * w[0] - zi * w[1];
                im += zr * w[1] + zi * w[0];
            }
            y[2 * (k1 + k2 * m)] = (double)re;
            y[2 * (k1 + k2 * m) + 1] = (double)im;
        }
    }
}

/*
 * The recursion above writes Z into `work` and uses y as the child's work area.
 * Both must hold n complex values; the child of size m only needs m of them,
 * and m * p = n, so the two buffers of size n suffice at every level.
 */
static void rec_1d_top(int64_t n, int sign, const double *x, int64_t xs, double *y, const ld *W)
{
    double *work = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    rec_1d(n, x, xs, y, W, n, work);
    free(work);
}

void oracle_fft_rec_1d(int64_t n, int sign, const double *x, int64_t xs, double *y)
{
    if (n <= 0) return;
    ld *W = root_table(n, sign);
    rec_1d_top(n, sign, x, xs, y, W);
    free(W);
}

/* ---------------------------------------------------------------- O3 */

typedef struct {
    int64_t n, M;
    ld *chirp;      /* c_k = exp(sign * pi i (k^2 mod 2n) / n), k < n           */
    ld *WMf, *WMi;  /* root tables of length M, forward (-1) and inverse (+1)    */
    double *vhat;   /* DFT_M of the wrapped conj(c) sequence                     */
} blue_t;

static void blue_init(blue_t *b, int64_t n, int sign)
{
    b->n = n;
    int64_t M = 1;
    while (M < 2 * n - 1) M <<= 1;
    b->M = M;
    b->chirp = (ld *)malloc(sizeof(ld) * 2 * n);
    for (int64_t k = 0; k < n; ++k) {
        int64_t q = (int64_t)(((__int128)k * k) % (2 * n));
        ld c, s;
        unit_root(q, 2 * n, &c, &s);             /* exp(2 pi i q / 2n) */
        b->chirp[2 * k] = c;
        b->chirp[2 * k + 1] = sign < 0 ? -s : s;
    }
    b->WMf = root_table(M, -1);
    b->WMi = root_table(M, +1);
    double *v = (double *)calloc(2 * (size_t)M, sizeof(double));
    for (int64_t k = 0; k < n; ++k) {
        v[2 * k] = (double)b->chirp[2 * k];
        v[2 * k + 1] = (double)-b->chirp[2 * k + 1];
        if (k > 0) {
            v[2 * (M - k)] = (double)b->chirp[2 * k];
            v[2 * (M - k) + 1] = (double)-b->chirp[2 * k + 1];
        }
    }
    b->vhat = (double *)malloc(sizeof(double) * 2 * M);
    rec_1d_top(M, -1, v, 1, b->vhat, b->WMf);
    free(v);
}

static void blue_free(blue_t *b)
{
    free(b->chirp);
    free(b->WMf);
    free(b->WMi);
    free(b->vhat);
}

/* Y[k] = c_k * (1/M) IDFT_M( DFT_M(u) * vhat )[k],  u_l = x_l c_l zero-padded. */
static void blue_apply(const blue_t *b, const double *x, int64_t xs, double *y)
{
    int64_t n = b->n, M = b->M;
    double *u = (double *)calloc(2 * (size_t)M, sizeof(double));
    double *U = (double *)malloc(sizeof(double) * 2 * M);
    for (int64_t l = 0; l < n; ++l) {
        ld xr = x[2 * l * xs], xi = x[2 * l * xs + 1];
        ld cr = b->chirp[2 * l], ci = b->chirp[2 * l + 1];
        u[2 * l] = (double)(xr * cr - xi * ci);
        u[2 * l + 1] = (double)(xr * ci + xi * cr);
    }
    rec_1d_top(M, -1, u, 1, U, b->WMf);
    for (int64_t k = 0; k < M; ++k) {
        ld ar = U[2 * k], ai = U[2 * k + 1];
        ld br = b->vhat[2 * k], bi = b->vhat[2 * k + 1];
        u[2 * k] = (double)(ar * br - ai * bi);
        u[2 * k + 1] = (double)(ar * bi + ai * br);
    }
    rec_1d_top(M, +1, u, 1, U, b->WMi);
    for (int64_t k = 0; k < n; ++k) {
        ld ar = U[2 * k] / (ld)M, ai = U[2 * k + 1] / (ld)M;
        ld cr = b->chirp[2 * k], ci = b->chirp[2 * k + 1];
        y[2 * k] = (double)(ar * cr - ai * ci);
        y[2 * k + 1] = (double)(ar * ci + ai * cr);
    }
    free(u);
    free(U);
}

void oracle_fft_bluestein_1d(int64_t n, int sign, const double *x, int64_t xs, double *y)
{
    if (n <= 0) return;
    blue_t b;
    blue_init(&b, n, sign);
    blue_apply(&b, x, xs, y);
    blue_free(&b);
}

/* ---------------------------------------------------------------- lines */

/* Per-length context for the separable driver: one root table (and Bluestein
 * state) per distinct length, built once before the worker threads start. */
typedef struct {
    int64_t n;
    int method;
    ld *W;
    blue_t blue;
    int has_blue;
} line_ctx;

static int is_prime64(int64_t n)
{
    if (n < 2) return 0;
    return smallest_factor(n) == n;
}

static void line_init(line_ctx *c, int64_t n, int sign, int method)
{
    memset(c, 0, sizeof(*c));
    c->n = n;
    if (method == OR_AUTO)
        method = (is_prime64(n) && n > 1024) ? OR_BLUESTEIN : OR_RECURSIVE;
    c->method = method;
    if (method == OR_BLUESTEIN) {
        blue_init(&c->blue, n, sign);
        c->has_blue = 1;
    } else {
        c->W = root_table(n, sign);
    }
}

static void line_free(line_ctx *c)
{
    free(c->W);
    if (c->has_blue) blue_free(&c->blue);
}

/* DFT of one contiguous line x (n complex) into y (n complex). */
static void line_apply(const line_ctx *c, const double *x, double *y, double *work)
{
    switch (c->method) {
    case OR_DIRECT: direct_1d(c->n, c->W, x, 1, y, 1); break;
    case OR_BLUESTEIN: blue_apply(&c->blue, x, 1, y); break;
    default: rec_1d(c->n, x, 1, y, c->W, c->n, work); break;
    }
}

/* ---------------------------------------------------------------- driver */

typedef struct {
    /* work array: V_total transforms, each a row-major block over N dims */
    double *buf;
    int64_t nv, ntot;
    int rank;
    int64_t shape[16];
    line_ctx *lines;      /* per dimension */
    int axis;
    int64_t nlines;       /* lines along `axis` over the whole work array */
    int nthreads;
} sep_job;

typedef struct {
    sep_job *job;
    int tid;
} sep_arg;

static void *sep_worker(void *p)
{
    sep_arg *a = (sep_arg *)p;
    sep_job *j = a->job;
    int ax = j->axis;
    int64_t n = j->shape[ax];
    int64_t inner = 1;                             /* stride of `axis` inside a block */
    for (int d = ax + 1; d < j->rank; ++d) inner *= j->shape[d];
    double *x = (double *)malloc(sizeof(double) * 2 * n);
    double *y = (double *)malloc(sizeof(double) * 2 * n);
    double *w = (double *)malloc(sizeof(double) * 2 * n);
    int64_t per = (j->nlines + j->nthreads - 1) / j->nthreads;
    int64_t lo = per * a->tid, hi = lo + per;
    if (hi > j->nlines) hi = j->nlines;
    for (int64_t L = lo; L < hi; ++L) {
        /* line L -> (outer block index, inner offset) */
        int64_t io = L % inner, oo = L / inner;
        double *base = j->buf + 2 * (oo * n * inner + io);
        for (int64_t l = 0; l < n; ++l) {
            x[2 * l] = base[2 * l * inner];
            x[2 * l + 1] = base[2 * l * inner + 1];
        }
        line_apply(&j->lines[ax], x, y, w);
        for (int64_t l = 0; l < n; ++l) {
            base[2 * l * inner] = y[2 * l];
            base[2 * l * inner + 1] = y[2 * l + 1];
        }
    }
    free(x);
    free(y);
    free(w);
    return NULL;
}

static void run_parallel(sep_job *job)
{
    int T = job->nthreads;
    if (T < 1) T = 1;
    if ((int64_t)T > job->nlines) T = (int)(job->nlines > 0 ? job->nlines : 1);
    job->nthreads = T;
    pthread_t th[256];
    sep_arg args[256];
    if (T > 256) T = job->nthreads = 256;
    for (int t = 0; t < T; ++t) {
        args[t].job = job;
        args[t].tid = t;
        if (t > 0) pthread_create(&th[t], NULL, sep_worker, &args[t]);
    }
    sep_worker(&args[0]);
    for (int t = 1; t < T; ++t) pthread_join(th[t], NULL);
}

/* offset of the element with multi-index idx[] along dims[] (input or output) */
static int64_t tensor_offset(const oracle_iodim *d, int r, const int64_t *idx, int out)
{
    int64_t off = 0;
    for (int i = 0; i < r; ++i) off += idx[i] * (out ? d[i].os : d[i].is);
    return off;
}

static int next_index(int64_t *idx, const oracle_iodim *d, int r)
{
    for (int i = r - 1; i >= 0; --i) {
        if (++idx[i] < d[i].n) return 1;
        idx[i] = 0;
    }
    return 0;
}

/*
 * Solve dft(N, V, I, O): `in` and `out` point at element (0,...,0) of the
 * tensors; strides are in complex elements (interleaved re, im doubles).
 * The caller guarantees every addressed element lies inside its buffer.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_dft(int rank, const oracle_iodim *dims, int vrank, const oracle_iodim *vdims,
               const double *in, double *out, int sign, int method, int nthreads)
{
    if (rank < 0 || rank > 16 || vrank < 0 || vrank > 16) return -1;
    if (sign != -1 && sign != 1) return -1;
    int64_t ntot = 1, nv = 1;
    for (int i = 0; i < rank; ++i) {
        if (dims[i].n < 0) return -1;
        ntot *= dims[i].n;
    }
    for (int i = 0; i < vrank; ++i) {
        if (vdims[i].n < 0) return -1;
        nv *= vdims[i].n;
    }
    if (ntot == 0 || nv == 0) return 0;          /* empty loop: nothing to do */

    /* snapshot: gather every transform into the work array before writing */
    double *buf = (double *)malloc(sizeof(double) * 2 * (size_t)(ntot * nv));
    if (!buf) return -1;
    int64_t vidx[16] = {0}, nidx[16] = {0};
    int64_t pos = 0;
    do {
        int64_t vin = tensor_offset(vdims, vrank, vidx, 0);
        memset(nidx, 0, sizeof(nidx));
        do {
            int64_t o = vin + tensor_offset(dims, rank, nidx, 0);
            buf[2 * pos] = in[2 * o];
            buf[2 * pos + 1] = in[2 * o + 1];
            ++pos;
        } while (rank > 0 && next_index(nidx, dims, rank));
    } while (vrank > 0 && next_index(vidx, vdims, vrank));

    if (method == OR_MD_DIRECT && rank > 0) {
        /* the multi-dimensional definition summed directly */
        ld *W[16];
        for (int d = 0; d < rank; ++d) W[d] = root_table(dims[d].n, sign);
        double *res = (double *)malloc(sizeof(double) * 2 * (size_t)ntot);
        for (int64_t v = 0; v < nv; ++v) {
            const double *x = buf + 2 * v * ntot;
            int64_t kidx[16] = {0};
            int64_t kpos = 0;
            do {
                ld re = 0.0L, im = 0.0L;
                int64_t lidx[16] = {0};
                int64_t lpos = 0;
                do {
                    ld wr = 1.0L, wi = 0.0L;
                    for (int d = 0; d < rank; ++d) {
                        int64_t e = (int64_t)(((__int128)lidx[d] * kidx[d]) % dims[d].n);
                        ld ar = W[d][2 * e], ai = W[d][2 * e + 1];
                        ld tr = wr * ar - wi * ai;
                        wi = wr * ai + wi * ar;
                        wr = tr;
                    }
                    ld xr = x[2 * lpos], xi = x[2 * lpos + 1];
                    re += xr * wr - xi * wi;
                    im += xr * wi + xi * wr;
                    ++lpos;
                } while (next_index(lidx, dims, rank));
                res[2 * kpos] = (double)re;
                res[2 * kpos + 1] = (double)im;
                ++kpos;
            } while (next_index(kidx, dims, rank));
            memcpy(buf + 2 * v * ntot, res, sizeof(double) * 2 * ntot);
        }
        free(res);
        for (int d = 0; d < rank; ++d) free(W[d]);
    } else if (rank > 0) {
        /* separable: 1D transforms along each dimension of each block */
        line_ctx lines[16];
        int lm = method == OR_MD_DIRECT ? OR_AUTO : method;
        for (int d = 0; d < rank; ++d) line_init(&lines[d], dims[d].n, sign, lm);
        sep_job job;
        memset(&job, 0, sizeof(job));
        job.buf = buf;
        job.nv = nv;
        job.ntot = ntot;
        job.rank = rank;
        for (int d = 0; d < rank; ++d) job.shape[d] = dims[d].n;
        job.lines = lines;
        for (int d = 0; d < rank; ++d) {
            if (dims[d].n == 1) continue;
            job.axis = d;
            job.nlines = nv * (ntot / dims[d].n);
            job.nthreads = nthreads;
            run_parallel(&job);
        }
        for (int d = 0; d < rank; ++d) line_free(&lines[d]);
    }

    /* scatter to the output tensor */
    memset(vidx, 0, sizeof(vidx));
    pos = 0;
    do {
        int64_t vout = tensor_offset(vdims, vrank, vidx, 1);
        memset(nidx, 0, sizeof(nidx));
        do {
            int64_t o = vout + tensor_offset(dims, rank, nidx, 1);
            out[2 * o] = buf[2 * pos];
            out[2 * o + 1] = buf[2 * pos + 1];
            ++pos;
        } while (rank > 0 && next_index(nidx, dims, rank));
    } while (vrank > 0 && next_index(vidx, vdims, vrank));
    free(buf);
    return 0;
}
