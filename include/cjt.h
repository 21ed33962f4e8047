/*
 * cjt.h -- C-ABI of the MI355X Chebyshev--Jacobi transform library (libcjt_hip.so).
 *
 * The transform pair (Slevinsky, "On the use of Hahn's asymptotic formula and
 * stabilized recurrence for a fast, simple, and stable Chebyshev--Jacobi
 * transform", IMA J. Numer. Anal.):
 *
 *   forward   c_cheb = T_N^{-1} P_N c_jac        (Sec. 1, eq. CJT)
 *   inverse   c_jac  = P_N^{-1} T_N c_cheb       (Sec. 1, eq. iCJT; computed by the
 *                                                 transposed formula, Sec. 3, eq. CJTT)
 *
 * where [P_N]_{j,n} = P_n^{(alpha,beta)}(x_j), [T_N]_{j,k} = T_k(x_j) and
 * x_j = cos(pi j / N), j = 0..N.  Both vectors hold N+1 doubles, index n (or k)
 * at offset n.
 *
 * The plan/execute split follows Sec. 4 (FFTW-like): cjt_plan computes the
 * partition of Sec. 2.2, the recurrence coefficients of Sec. 1.2 and 4.2, the
 * Hahn diagonals of Sec. 2.1 and, for the inverse, the Clenshaw--Curtis
 * weights and orthonormality constants of Sec. 3; execution applies them.
 *
 * Conventions for every entry point:
 *   - Device pointers ("d_") are HIP device addresses on the device that is
 *     current when the plan was created; host pointers are ordinary memory.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Execution calls are
 *     asynchronous on that stream; argument errors are returned synchronously
 *     and nothing is launched.  A stream is used by one call at a time: the
 *     library keeps one workspace per stream.
 *   - Plans are immutable after creation and may be used from several streams;
 *     the caller owns every input and output buffer, the plan owns its device
 *     arrays.  Out-of-place only: d_in == d_out returns CJT_EINVAL.
 *   - On error, cjt_last_error() returns a message for the calling thread.
 */
#ifndef CJT_H
#define CJT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cjt_plan_s* cjt_plan_t;
typedef struct cjt_batch_s* cjt_batch_t;

typedef enum {
    CJT_OK = 0,
    CJT_EINVAL = 1,      /* bad size, pointer or flag */
    CJT_EDOMAIN = 2,     /* alpha or beta outside (-1/2, 1/2] (Sec. 2.1), or M outside {0} U [2, 30] */
    CJT_ENOMEM = 3,      /* device or host allocation failed */
    CJT_EDEVICE = 4,     /* a HIP call failed */
    CJT_EBUSY = 5,       /* resource in use */
    CJT_EUNSUPPORTED = 6, /* valid request this build does not implement */
    CJT_ECANCELED = 7     /* serving: the request was cancelled before it ran */
} cjt_status;

/* Plan flags. */
enum {
    CJT_FP64 = 0,          /* every step in FP64 */
    CJT_FP32_BULK = 1,     /* the DCT-I/DST-I of the Hahn blocks in FP32 with FP32 accumulation;
                              diagonals, recurrences and boundary DCTs stay FP64 */
    CJT_BATCH_INVARIANT = 8, /* results of this plan are bitwise the same whatever else shares a
                              batched call: its recurrence segments are sized from its own
                              degree alone instead of from the whole batch */
    CJT_SHIFT = 16          /* parameters -1 < alpha, beta <= 5/2: the core runs at the integer
                              shift (alpha0, beta0) in (-1/2, 1/2]^2 and the coefficients are
                              carried between the two families by the relation between
                              neighbouring parameters (Sec. 1.2), O(N) per unit of shift.  The
                              inverse's error grows like N^s for s unit shifts up (the paper's
                              remark on large parameters), hence the cap.  Not for servers or
                              persistent batches */
};

/* Direction flags of a persistent batch. */
enum {
    CJT_DIR_FWD = 2,       /* forward transforms (eq. CJT) */
    CJT_DIR_INV = 4        /* inverse transforms (eq. CJTT) */
};

#define CJT_MAX_BLOCKS 16

/* Partition of Sec. 2.2 for one grid: nblocks rectangles
 * [win_lo[k], win_hi[k]] (grid indices, inclusive) x [deg_lo[k], deg_hi[k])
 * (degrees, half-open) where Hahn's expansion with M terms is within eps;
 * everything else is evaluated by recurrence. */
typedef struct {
    int64_t grid;            /* number of intervals G: points are cos(pi i / G), i = 0..G */
    int32_t M;               /* terms used */
    int32_t nblocks;         /* K' <= K */
    int64_t n_M;             /* eq. for n_M, with the envelope g_M(pi/2) */
    double alpha_N;          /* min(1/log(G/n_M), 1/2) */
    int32_t K;               /* ceil(log(G/n_M)/log(1/alpha_N)) */
    int32_t theta_bar;       /* grid index of the discrete minimiser of g_M */
    int64_t deg_lo[CJT_MAX_BLOCKS], deg_hi[CJT_MAX_BLOCKS];
    int64_t win_lo[CJT_MAX_BLOCKS], win_hi[CJT_MAX_BLOCKS];
    int64_t rec_entries;     /* number of (point, degree) pairs left to recurrence */
} cjt_partition_info;

typedef struct {
    int64_t N;
    double alpha, beta;
    int32_t M;               /* Hahn terms in use (chosen when 0 was requested) */
    uint32_t flags;
    double eps;              /* partition tolerance, 2^-52 */
    cjt_partition_info fwd;  /* grid N, degrees 0..N */
    cjt_partition_info inv;  /* grid 2N, degrees clipped to 0..N (Sec. 3.2) */
    int64_t fft_len_fwd;     /* complex FFT length behind one DCT-I + DST-I pair: N */
    int64_t fft_len_inv;     /* 2N */
    int64_t fft_count_fwd;   /* Hahn-block transforms per forward call: M x nblocks */
    int64_t fft_count_inv;
    size_t device_bytes;     /* device memory held by the plan */
    int32_t fft_log2_cols_fwd; /* two-pass split of the forward FFTs: log2 of the column length (0: one pass) */
    int32_t fft_log2_cols_inv; /* the same for the inverse's length-2N FFTs */
    int32_t shift_alpha;     /* CJT_SHIFT: alpha - alpha0 (integer), else 0 */
    int32_t shift_beta;      /* beta - beta0 */
} cjt_plan_info;

/* Create a plan for degree 1 <= N <= 2^21 (larger N return CJT_EUNSUPPORTED;
 * lengths that are not powers of two run their FFTs as chirp-z convolutions),
 * parameters (alpha, beta) in (-1/2, 1/2]
 * (Sec. 2.1: Hahn's remainder bound), and M Hahn terms (0 = chosen by the
 * library's cost model, else 2 <= M <= 30; Sec. 2.2 needs M >= 2).  flags is
 * CJT_FP64 or CJT_FP32_BULK, optionally or-ed with CJT_BATCH_INVARIANT.  Plan arrays are computed on the device on
 * `stream`; the call returns after they are complete.  *out receives the plan. */
cjt_status cjt_plan(cjt_plan_t* out, int64_t N, double alpha, double beta, int M, unsigned flags,
                    void* stream);

/* Forward transform (eq. CJT): d_in = Jacobi coefficients c_0..c_N, d_out =
 * Chebyshev coefficients, N+1 doubles each, device memory, no overlap. */
cjt_status cjt_forward(cjt_plan_t plan, const double* d_in, double* d_out, void* stream);

/* Inverse transform (eq. iCJT via eq. CJTT): d_in = Chebyshev coefficients,
 * d_out = Jacobi coefficients, N+1 doubles each, device memory, no overlap. */
cjt_status cjt_inverse(cjt_plan_t plan, const double* d_in, double* d_out, void* stream);

/* Batched forward/inverse: `count` independent transforms, transform i uses
 * plans[i] (a host array; plans may repeat) and the ragged slices
 * d_in[offsets[i] .. offsets[i+1]) and d_out[same], where offsets is a host
 * array of count+1 entries with offsets[i+1] - offsets[i] = N_i + 1.  All
 * plans must share one precision flag.  One launch sequence serves the whole
 * batch, whatever the mix of degrees: each kernel runs over a flat list of
 * work items of all instances. */
cjt_status cjt_forward_batched(const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                               const double* d_in, double* d_out, void* stream);
cjt_status cjt_inverse_batched(const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                               const double* d_in, double* d_out, void* stream);

/* Jacobi-to-Jacobi transform by composition (Conclusions: the forward
 * transform followed by the inverse one changes the parameters of an
 * expansion): d_out = inverse_to(forward_from(d_in)), so that
 * sum_n d_in[n] P_n^(a,b) = sum_n d_out[n] P_n^(c,d) with (a, b) the
 * parameters of `from` and (c, d) those of `to`.  Both plans have the same
 * N and precision flag; d_in and d_out hold N+1 doubles each in device memory
 * and must not overlap.  The Chebyshev coefficients in between live in a
 * buffer the library keeps per device and stream (grown on demand, which
 * synchronizes the stream once).  Errors: CJT_EINVAL for null or overlapping
 * buffers, differing N or precision; otherwise those of cjt_forward and
 * cjt_inverse. */
cjt_status cjt_jacobi_to_jacobi(cjt_plan_t from, cjt_plan_t to, const double* d_in, double* d_out, void* stream);

/* Batched Jacobi-to-Jacobi: transform i uses from[i] and to[i] (host arrays,
 * from[i] and to[i] of the same N) on the ragged slices given by offsets, as
 * in cjt_forward_batched; one batched forward and one batched inverse. */
cjt_status cjt_jacobi_to_jacobi_batched(const cjt_plan_t* from, const cjt_plan_t* to, int64_t count,
                                        const int64_t* offsets, const double* d_in, double* d_out, void* stream);

/* Persistent batch (Sec. 4: many sets of coefficients, one plan each).
 * cjt_batch_create does all host-side work once: it lays out the launch
 * program for `count` transforms (plans[i], ragged slices given by the host
 * array offsets as in cjt_forward_batched; flags = CJT_DIR_FWD or
 * CJT_DIR_INV), allocates the batch's own device workspace (FFT
 * intermediates of every instance at once, so no chunking), and uploads the
 * descriptors and work items; it returns when they are resident.  The plans
 * must outlive the batch.  cjt_batch_execute only launches kernels on
 * `stream` and on a stream the batch owns (joined back before it returns), so
 * a call can be captured into a HIP graph and replayed; d_in / d_out are
 * the base pointers of the ragged arrays (any pointers on each call).  Calls
 * on one batch must not overlap in time: they share its workspace. */
typedef struct {
    int64_t count;            /* transforms */
    int64_t launches;         /* kernel launches per execution (plus stream fork/join) */
    int64_t items;            /* work items over all launches */
    size_t workspace_bytes;   /* device memory held by the batch besides descriptors */
    int32_t inverse;          /* 1 for CJT_DIR_INV */
} cjt_batch_info;

cjt_status cjt_batch_create(cjt_batch_t* out, const cjt_plan_t* plans, int64_t count, const int64_t* offsets,
                            unsigned flags, void* stream);
cjt_status cjt_batch_execute(cjt_batch_t batch, const double* d_in, double* d_out, void* stream);
cjt_status cjt_batch_query(cjt_batch_t batch, cjt_batch_info* out);
/* Release a batch (waits for the device). NULL is accepted. */
cjt_status cjt_batch_destroy(cjt_batch_t batch);

/* ------------------------------------------------------------------ serving
 *
 * A transform server (Sec. 4: plans made once and reused for many sets of
 * coefficients) for a stream of independent requests of any degree,
 * direction and parameters, on one device.  A batcher thread takes the
 * queued requests of one direction and precision (oldest first, at most
 * max_batch) and issues them as one batched call while earlier calls still
 * run (continuous batching: at most max_inflight calls queued on the device);
 * a completion thread stamps each request's latency (arrival to completion of
 * its call, host clock) when the call's event completes.
 *
 * Memory: the server allocates its whole HBM budget once at creation and
 * never more.  It holds the execution workspace (workspace_bytes), one
 * descriptor buffer of max(16 MiB, max_batch x 256 KiB) per call in flight
 * (a call whose work items do not fit is split), and resident plans keyed by
 * (N, alpha, beta, precision), least recently used first out when a new plan
 * does not fit; a plan used by a queued or running call is never evicted.
 * A request whose plan or workspace cannot fit even in an empty server fails
 * with CJT_ENOMEM; one that waits for memory held by running calls is
 * admitted when they complete.  The power-of-two FFT twiddle tables are
 * shared library-wide and are not part of the budget.
 *
 * Requests: flags = CJT_DIR_FWD or CJT_DIR_INV, optionally | CJT_FP32_BULK;
 * d_in / d_out are device buffers of N + 1 doubles that stay valid and
 * untouched until the request completes, and d_in must be ready when the
 * request is submitted.  Server plans are made with CJT_BATCH_INVARIANT, so a
 * result is bitwise the result of the same request executed alone with such
 * a plan, whatever it was batched with. */
typedef struct cjt_server_s* cjt_server_t;

typedef struct {
    size_t hbm_budget;        /* device bytes the server may hold (required) */
    size_t workspace_bytes;   /* part of the budget for execution intermediates (0: a quarter) */
    int32_t max_batch;        /* requests per batched call (0: 256) */
    int32_t max_inflight;     /* batched calls queued on the device at once (0: 2) */
    int32_t M;                /* Hahn terms of new plans (0: the cost model's choice) */
    int32_t start_paused;     /* 1: the batcher takes no request until cjt_server_pause(s, 0) */
} cjt_server_config;

typedef struct {
    int64_t submitted, completed, failed, cancelled;
    int64_t batches;              /* batched calls issued */
    double mean_batch;            /* requests per batched call */
    int64_t plan_hits, plan_misses, plan_evictions;
    int64_t admission_stalls;     /* times the batcher waited for memory held by running calls */
    int64_t plans_resident;
    size_t plan_bytes;            /* device bytes of resident plans */
    size_t budget_bytes;          /* the server's allocation (= hbm_budget) */
    size_t peak_used_bytes;       /* high-water mark of budget bytes in use */
    int64_t lat_count;            /* completed requests since the last reset */
    double lat_p50_us, lat_p99_us, lat_mean_us, lat_max_us;
} cjt_server_stats;

/* Create a server on the current device; allocates the budget.  CJT_EINVAL
 * if the budget cannot hold the workspace and descriptor buffers. */
cjt_status cjt_server_create(cjt_server_t* out, const cjt_server_config* cfg);
/* Queue one request (arrival = now).  Argument errors return synchronously
 * and queue nothing; *ticket identifies the request. */
cjt_status cjt_server_submit(cjt_server_t s, unsigned flags, int64_t N, double alpha, double beta,
                             const double* d_in, double* d_out, int64_t* ticket);
/* Load generator: submits request i (host arrays of `count` entries) at
 * arrival_us[i] microseconds after the call starts (non-decreasing), waiting
 * on the host clock in between; latency counts from that scheduled arrival.
 * Returns after the last submission.  A request with bad arguments gets
 * ticket -1 and is counted as failed. */
cjt_status cjt_server_replay(cjt_server_t s, int64_t count, const unsigned* flags, const int64_t* N,
                             const double* alpha, const double* beta, const double* const* d_in,
                             double* const* d_out, const double* arrival_us, int64_t* tickets);
/* Block until the request completes; *result receives its status (CJT_OK,
 * CJT_ENOMEM, CJT_EDEVICE, CJT_ECANCELED, ...), *latency_us its latency
 * (either may be NULL).  The ticket is then forgotten. */
cjt_status cjt_server_wait(cjt_server_t s, int64_t ticket, cjt_status* result, double* latency_us);
/* Cancel a request still in the queue: CJT_OK (its result becomes
 * CJT_ECANCELED), CJT_EBUSY if it was already taken into a call. */
cjt_status cjt_server_cancel(cjt_server_t s, int64_t ticket);
/* Stop (1) or resume (0) taking requests from the queue. */
cjt_status cjt_server_pause(cjt_server_t s, int paused);
/* Block until every submitted request has completed (not while paused with
 * requests queued: returns CJT_EBUSY then). */
cjt_status cjt_server_drain(cjt_server_t s);
/* Counters and latency percentiles; reset != 0 clears the latency record
 * and the counters after reading. */
cjt_status cjt_server_query(cjt_server_t s, cjt_server_stats* out, int reset);
/* Drain, stop the threads and release everything. NULL is accepted. */
cjt_status cjt_server_destroy(cjt_server_t s);

/* ------------------------------------------------------------------ schedule autotuner
 *
 * FFTs longer than 4096 points run in two passes, L = L1 x L2 (column FFTs of
 * length L1, row FFTs of length L2; chirp-z transforms split their
 * power-of-two convolution length P the same way).  The split is a schedule
 * choice: it changes occupancy and memory transactions, not the transform.
 * The library keeps a table of splits keyed by (power-of-two length,
 * inverse, chirp-z, precision); plans read it when they are created and keep
 * the split they were made with.  Untuned lengths use L1 = 2^floor(lg/2).
 * If CJT_TUNE_FILE names a file, it is loaded on first use. */
typedef struct {
    int64_t fft_len;            /* power-of-two length tuned (L, or P for chirp-z) */
    int32_t inverse, chirp, fp32;
    int32_t candidates;         /* splits timed */
    int32_t log2_cols_default;  /* split before tuning */
    int32_t log2_cols_best;     /* split now in the table */
    double ms_default, ms_best; /* mean time of one batched call with each */
} cjt_tune_entry;

/* Times every accepted split of the two-pass FFTs that a plan of degree N
 * uses (forward length N, inverse length 2N; lengths up to 4096 need none)
 * on a synthetic plan (alpha = beta = 0.1, automatic M, the precision of
 * `flags`: CJT_FP64 or CJT_FP32_BULK): `reps` batched calls of `batch`
 * (1..4096) transforms of each direction per candidate on `stream`; stores the
 * fastest in the table.  out receives one entry per tuned length (at most 2;
 * *n_out of them).  Allocates and frees its own device buffers; returns after
 * the device work completed. */
cjt_status cjt_autotune(int64_t N, unsigned flags, int64_t batch, int reps, void* stream, cjt_tune_entry* out,
                        int* n_out);
/* Set one table entry (log2_cols = -1 removes it).  CJT_EINVAL for a length
 * that runs in one pass or a split outside [max(4, lg-11), min(11, lg-4)]. */
cjt_status cjt_tune_set(int64_t fft_len, int inverse, int chirp, int fp32, int log2_cols);
/* Write / merge the table as text, one entry per line:
 * "fft_len inverse chirp fp32 log2_cols" ('#' starts a comment).  Host only. */
cjt_status cjt_tune_save(const char* path);
cjt_status cjt_tune_load(const char* path);

/* Describe a plan (host memory out). */
cjt_status cjt_plan_query(cjt_plan_t plan, cjt_plan_info* out);

/* Host-only: the plan summary cjt_plan would build (partitions, chosen M,
 * transform counts), without touching a device.  device_bytes is an estimate. */
cjt_status cjt_plan_describe(int64_t N, double alpha, double beta, int M, unsigned flags, cjt_plan_info* out);

/* Release a plan (waits for the device to finish with it). NULL is accepted. */
cjt_status cjt_plan_destroy(cjt_plan_t plan);

/* Static text for a status code. */
const char* cjt_strerror(cjt_status status);

/* Detail message of the last error on the calling thread ("" if none). */
const char* cjt_last_error(void);

/* Kernel timing (instrumentation).  While enabled, every kernel launch of the
 * execution calls is bracketed by HIP events recorded on the caller's stream,
 * and tagged with the algorithmic work of that launch: floating-point
 * operations by a fixed convention (2.5 L log2 L per real FFT of length L,
 * i.e. per DCT-I + DST-I pair of a Hahn block, plus 4 per diagonal scaling of
 * a window point and 2 per coefficient scaling; 6 per three-term or
 * Clenshaw--Smith step and 10 per modified step of Sec. 4.2) and the
 * compulsory HBM bytes (each vector the kernel must read or write, once).  cjt_profile_collect waits for the
 * device, sums time and work per kernel name into out[0 .. *n_out) (at most
 * max entries) and clears the record.  Timing adds two event records per
 * launch; leave it off outside measurement. */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
    double flops;        /* algorithmic flops over all launches */
    double bytes;        /* compulsory HBM bytes over all launches */
} cjt_kernel_stat;

cjt_status cjt_profile_enable(int on);
cjt_status cjt_profile_collect(cjt_kernel_stat* out, int max, int* n_out);

/* Library version, as major*10000 + minor*100 + patch. */
int cjt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CJT_H */
