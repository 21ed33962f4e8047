/*
 * Plain CPU oracle for the Chebyshev--Jacobi transform (CJT).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: it is used by tests/, by __graft_entry__.smoke() to check
 * one GPU result, and by the cpu_baseline leg of bench.py.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * What it computes (Slevinsky, "On the use of Hahn's asymptotic formula and
 * stabilized recurrence for a fast, simple, and stable Chebyshev--Jacobi
 * transform", IMA J. Numer. Anal.):
 *
 *   forward   c_cheb = T_N^{-1} P_N c_jac                      (Sec. 1, eq. CJT)
 *   inverse   c_jac  = P_N^{-1} T_N c_cheb                     (Sec. 1, eq. iCJT)
 *
 * with [P_N]_{j,n} = P_n^{(a,b)}(x_j), [T_N]_{j,k} = T_k(x_j) and
 * x_j = cos(pi j / N), j = 0..N (Sec. 1, Chebyshev--Lobatto points).
 *
 * The forward transform is the definition written out: every point value
 * p_j = sum_n c_n P_n(x_j) comes from the three-term recurrence of Sec. 1.2,
 * then T_N^{-1} is applied as a direct O(N^2) sum (T_N is a diagonally scaled
 * DCT-I, Sec. 2).  The inverse is the exact weighted projection of Sec. 3
 * (eqs. cjintdefn, Anab, CCweights, CJTT): p_N is evaluated at the 2N+1
 * Chebyshev--Lobatto points, multiplied by the Clenshaw--Curtis weights of the
 * Jacobi weight (exact for degree <= 2N), projected onto each P_n by direct
 * summation, and divided by the orthonormality constants.  No asymptotics, no
 * partition, no FFT: every sum is a plain O(N^2) loop.
 *
 * Arithmetic: 80-bit long double throughout (64-bit significand); outputs are
 * rounded to double once at the end.  Built with -DORACLE_QUAD the same file
 * runs in binary128 with the unmodified recurrence everywhere; tests use that
 * build to check the long double one.  Readings where the paper is silent or
 * inconsistent:
 *   - the first modified moment is mu_1 = (b-a)/(a+b+2) mu_0; the printed
 *     (a-b) has the wrong sign (integrate x (1-x)^a (1+x)^b by parts);
 *   - A_0 = (a+b+2)/2, B_0 = (a-b)/2 (the printed forms are 0/0 at a+b = 0
 *     or -1), and the n = 0 normalisation uses (a+b+1)Gamma(a+b+1) =
 *     Gamma(a+b+2);
 *   - A_n x + B_n is evaluated as A_n (x - x0) + (A_n x0 + B_n) with x0 the
 *     nearer endpoint and x - 1 = -2 sin^2(theta/2), x + 1 = 2 cos^2(theta/2),
 *     the accurate forms the paper uses for x -/+ 1 (Sec. 4.2), and for
 *     theta <= pi/4 or >= 3pi/4 the recurrence is run in the paper's
 *     algebraically identical modified form (Sec. 4.2).  The printed form loses
 *     accuracy like n^2 eps next to x = +-1 (about 4e-13 at n = 4096 in long
 *     double), which would otherwise dominate the oracle's own error.
 *
 * Threads only split independent outputs (rows, degrees, or fixed blocks of
 * points reduced in a fixed order), so results do not depend on the thread
 * count.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_QUAD
/* Cross-check build: binary128 arithmetic and the plain three-term recurrence
 * at every point (no endpoint rewrite). */
#include <quadmath.h>
typedef __float128 real;
#define RSIN sinq
#define RFABS fabsq
#define REXP expq
#define RPOW powq
#define RLGAMMA lgammaq
#define PI_LIT 3.141592653589793238462643383279502884Q
#define USE_ENDPOINT_FORM 0
#else
typedef long double real;
#define RSIN sinl
#define RFABS fabsl
#define REXP expl
#define RPOW powl
#define RLGAMMA lgammal
#define PI_LIT 3.141592653589793238462643383279502884L
#define USE_ENDPOINT_FORM 1
#endif

#define ORACLE_OK 0
#define ORACLE_EINVAL 1
#define ORACLE_ENOMEM 3

static const real PI_L = PI_LIT;

/* ---------------------------------------------------------------- helpers */

/* cos(pi * r / d) for an integer r, reduced to a small argument first. */
static real cospi_frac(int64_t r, int64_t d)
{
    /* period 2d */
    int64_t p = 2 * d;
    r %= p;
    if (r < 0) r += p;
    if (r > d) r = p - r;          /* cos is even about 0 and pi */
    /* r in [0, d]: cos(pi r/d) = sin(pi (d - 2r) / (2d)) */
    real t = PI_L * (real)(d - 2 * r) / (real)(2 * d);
    return RSIN(t);
}

/* sin(pi * r / d) for integer r, via the cosine of the complementary angle. */
static real sinpi_frac(int64_t r, int64_t d)
{
    /* sin(pi r/d) = cos(pi (d - 2r) / (2d)) */
    return cospi_frac(d - 2 * r, 2 * d);
}

/* Neumaier compensated accumulator. */
typedef struct { real s, c; } acc_t;
static inline void acc_add(acc_t* a, real v)
{
    real t = a->s + v;
    if (RFABS(a->s) >= RFABS(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}
static inline real acc_get(const acc_t* a) { return a->s + a->c; }

/* Recurrence coefficients of Sec. 1.2 (DLMF 18.9.2), for n >= 0, plus the
 * endpoint ratios r_n(+-1) = P_{n+1}(+-1) / P_n(+-1) of Sec. 4.2, which follow
 * from the endpoint values binom(n+a, n) and (-1)^n binom(n+b, n). */
typedef struct { real A, B, C, rp, rm, sp, sm; } rec_t;

static void rec_coeffs(int64_t nmax, real a, real b, rec_t* out)
{
    for (int64_t n = 0; n <= nmax; ++n) {
        real nn = (real)n;
        if (n == 0) {
            out[0].A = (a + b + 2.0L) / 2.0L;
            out[0].B = (a - b) / 2.0L;
            out[0].C = 0.0L; /* multiplies P_{-1} = 0 */
        } else {
            real s = 2.0L * nn + a + b;
            out[n].A = (s + 1.0L) * (s + 2.0L) / (2.0L * (nn + 1.0L) * (nn + a + b + 1.0L));
            out[n].B = (a - b) * (a + b) * (s + 1.0L) / (2.0L * (nn + 1.0L) * (nn + a + b + 1.0L) * s);
            out[n].C = (nn + a) * (nn + b) * (s + 2.0L) / ((nn + 1.0L) * (nn + a + b + 1.0L) * s);
        }
        out[n].rp = (nn + a + 1.0L) / (nn + 1.0L);
        out[n].rm = -(nn + b + 1.0L) / (nn + 1.0L);
        out[n].sp = out[n].A + out[n].B;   /* A_n x0 + B_n at x0 = +1 */
        out[n].sm = -out[n].A + out[n].B;  /* and at x0 = -1 */
    }
}

/* Evaluation of P_0, P_1, ... at theta = pi j / d, x = cos(theta).
 *
 * x - x0 is taken from the half-angle forms x - 1 = -2 sin^2(theta/2) and
 * x + 1 = 2 cos^2(theta/2) with x0 the nearer endpoint, so the rounding of x
 * itself never enters.  Then:
 *   mode 0:  P_{n+1} = (A_n (x - x0) + (A_n x0 + B_n)) P_n - C_n P_{n-1}, the
 *            three-term recurrence as printed with A_n x + B_n regrouped;
 *   mode +1/-1 (theta <= pi/4, resp. >= 3pi/4; long double build only): the
 *            same recurrence after substituting B_n = r_n + C_n / r_{n-1} - A_n x0
 *            (Sec. 4.2, modified forward recurrence):
 *              d_{n+1} = (A_n (x - x0) P_n + C_n d_n) / r_n,
 *              P_{n+1} = (P_n + d_{n+1}) r_n,      d_0 = 0.
 * In exact arithmetic both give P_n; near x = +-1 the first loses accuracy
 * like n^2 eps, which the second avoids.  The binary128 build uses mode 0
 * everywhere and checks this one. */
typedef struct {
    int mode;     /* 0, +1, -1 */
    int side;     /* x0 = +1 or -1 */
    real dx;      /* x - x0 */
    real p, pm1, d;
} walker_t;

static void walker_init(walker_t* w, int64_t j, int64_t d)
{
    /* theta/2 = pi j / (2d) */
    if (2 * j <= d) {
        real s = sinpi_frac(j, 2 * d);
        w->dx = -2.0L * s * s;
        w->side = +1;
    } else {
        real c = cospi_frac(j, 2 * d);
        w->dx = 2.0L * c * c;
        w->side = -1;
    }
    w->mode = 0;
    if (USE_ENDPOINT_FORM) {
        if (4 * j <= d) w->mode = +1;
        else if (4 * j >= 3 * d) w->mode = -1;
    }
    w->p = 1.0L;
    w->pm1 = 0.0L;
    w->d = 0.0L;
}

/* Advance from P_n to P_{n+1}. */
static inline void walker_step(walker_t* w, const rec_t* rc, int64_t n)
{
    const rec_t* c = &rc[n];
    if (w->mode == 0) {
        real shift = w->side > 0 ? c->sp : c->sm;
        real p1 = (c->A * w->dx + shift) * w->p - c->C * w->pm1;
        w->pm1 = w->p;
        w->p = p1;
    } else {
        real r = w->mode > 0 ? c->rp : c->rm;
        real d1 = (c->A * w->dx * w->p + c->C * w->d) / r;
        w->d = d1;
        w->p = (w->p + d1) * r;
    }
}

/* ------------------------------------------------------------- threading */

typedef void (*range_fn)(int64_t lo, int64_t hi, void* ctx);
typedef struct {
    range_fn fn;
    void* ctx;
    int64_t total;
    int64_t chunk;
    int64_t next;
    pthread_mutex_t mu;
} pool_t;

static void* pool_worker(void* arg)
{
    pool_t* p = (pool_t*)arg;
    for (;;) {
        pthread_mutex_lock(&p->mu);
        int64_t lo = p->next;
        p->next += p->chunk;
        pthread_mutex_unlock(&p->mu);
        if (lo >= p->total) break;
        int64_t hi = lo + p->chunk;
        if (hi > p->total) hi = p->total;
        p->fn(lo, hi, p->ctx);
    }
    return NULL;
}

static void run_parallel(int64_t total, int64_t chunk, int nthreads, range_fn fn, void* ctx)
{
    if (nthreads < 1) nthreads = 1;
    if (chunk < 1) chunk = 1;
    pool_t p;
    p.fn = fn; p.ctx = ctx; p.total = total; p.chunk = chunk; p.next = 0;
    pthread_mutex_init(&p.mu, NULL);
    if (nthreads == 1) {
        pool_worker(&p);
    } else {
        pthread_t* th = (pthread_t*)malloc(sizeof(pthread_t) * (size_t)nthreads);
        int started = 0;
        for (int t = 0; t < nthreads; ++t)
            if (pthread_create(&th[t], NULL, pool_worker, &p) == 0) ++started;
        if (started == 0) pool_worker(&p);
        for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
        free(th);
    }
    pthread_mutex_destroy(&p.mu);
}

/* -------------------------------------------- Jacobi values at grid points */

/* P_n^{(a,b)}(cos(pi j / d)) for n = 0..nmax, by the three-term recurrence. */
int oracle_jacobi_column(int64_t nmax, double alpha, double beta, int64_t j, int64_t d, double* out)
{
    if (nmax < 0 || d < 1 || j < 0 || j > d || !out) return ORACLE_EINVAL;
    real a = alpha, b = beta;
    rec_t* rc = (rec_t*)malloc(sizeof(rec_t) * (size_t)(nmax + 1));
    if (!rc) return ORACLE_ENOMEM;
    rec_coeffs(nmax, a, b, rc);
    walker_t w;
    walker_init(&w, j, d);
    for (int64_t n = 0; n <= nmax; ++n) {
        out[n] = (double)w.p;
        walker_step(&w, rc, n);
    }
    free(rc);
    return ORACLE_OK;
}

/* ------------------------------------------------------------- forward */

typedef struct {
    int64_t N;
    const rec_t* rc;
    const double* c;
    const int64_t* rows; /* NULL: all rows 0..N */
    real* p;             /* point values, long double */
} pv_ctx;

static void pv_range(int64_t lo, int64_t hi, void* vctx)
{
    pv_ctx* x = (pv_ctx*)vctx;
    int64_t N = x->N;
    for (int64_t r = lo; r < hi; ++r) {
        int64_t j = x->rows ? x->rows[r] : r;
        walker_t w;
        walker_init(&w, j, N);
        acc_t s = {0.0L, 0.0L};
        for (int64_t n = 0; n <= N; ++n) {
            acc_add(&s, (real)x->c[n] * w.p);
            if (n == N) break;
            walker_step(&w, x->rc, n);
        }
        x->p[r] = acc_get(&s);
    }
}

typedef struct {
    int64_t N;
    const real* p;
    const real* costab; /* cos(pi r / N), r = 0..2N-1 */
    double* out;
} dct_ctx;

/* c_k = (2/N)(1 - (d_k0 + d_kN)/2) sum_j (1 - (d_j0 + d_jN)/2) p_j cos(pi j k / N):
 * the inverse of [T_N]_{j,k} = cos(pi j k / N), written out. */
static void dct_range(int64_t lo, int64_t hi, void* vctx)
{
    dct_ctx* x = (dct_ctx*)vctx;
    int64_t N = x->N, P = 2 * N;
    for (int64_t k = lo; k < hi; ++k) {
        acc_t s = {0.0L, 0.0L};
        int64_t r = 0;
        for (int64_t j = 0; j <= N; ++j) {
            real wj = (j == 0 || j == N) ? 0.5L : 1.0L;
            acc_add(&s, wj * x->p[j] * x->costab[r]);
            r += k;
            if (r >= P) r -= P;
        }
        real wk = (k == 0 || k == N) ? 0.5L : 1.0L;
        x->out[k] = (double)(2.0L / (real)N * wk * acc_get(&s));
    }
}

static int forward_impl(int64_t N, double alpha, double beta, const double* c, double* out,
                        double* pvals, int nthreads)
{
    if (N < 1 || !c || (!out && !pvals)) return ORACLE_EINVAL;
    if (!(alpha > -1.0) || !(beta > -1.0)) return ORACLE_EINVAL;
    real a = alpha, b = beta;
    rec_t* rc = (rec_t*)malloc(sizeof(rec_t) * (size_t)(N + 1));
    real* p = (real*)malloc(sizeof(real) * (size_t)(N + 1));
    real* ct = (real*)malloc(sizeof(real) * (size_t)(2 * N));
    if (!rc || !p || !ct) { free(rc); free(p); free(ct); return ORACLE_ENOMEM; }
    rec_coeffs(N, a, b, rc);
    pv_ctx pc = {N, rc, c, NULL, p};
    run_parallel(N + 1, 16, nthreads, pv_range, &pc);
    if (pvals)
        for (int64_t j = 0; j <= N; ++j) pvals[j] = (double)p[j];
    if (out) {
        for (int64_t r = 0; r < 2 * N; ++r) ct[r] = cospi_frac(r, N);
        dct_ctx dc = {N, p, ct, out};
        run_parallel(N + 1, 16, nthreads, dct_range, &dc);
    }
    free(rc); free(p); free(ct);
    return ORACLE_OK;
}

/* Forward CJT: out[k], k = 0..N, from c[n], n = 0..N (eq. CJT). */
int oracle_forward(int64_t N, double alpha, double beta, const double* c, double* out, int nthreads)
{
    return forward_impl(N, alpha, beta, c, out, NULL, nthreads);
}

/* Point values p_j = sum_n c_n P_n(x_j), j = 0..N (the vector P_N c of eq. PTNPN). */
int oracle_point_values(int64_t N, double alpha, double beta, const double* c, double* p, int nthreads)
{
    return forward_impl(N, alpha, beta, c, NULL, p, nthreads);
}

/* Point values at selected rows only (O(N) per row), for spot checks at large N. */
int oracle_point_values_rows(int64_t N, double alpha, double beta, const double* c,
                             int64_t nrows, const int64_t* rows, double* p, int nthreads)
{
    if (N < 1 || !c || !rows || !p || nrows < 0) return ORACLE_EINVAL;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] > N) return ORACLE_EINVAL;
    real a = alpha, b = beta;
    rec_t* rc = (rec_t*)malloc(sizeof(rec_t) * (size_t)(N + 1));
    real* pl = (real*)malloc(sizeof(real) * (size_t)(nrows > 0 ? nrows : 1));
    if (!rc || !pl) { free(rc); free(pl); return ORACLE_ENOMEM; }
    rec_coeffs(N, a, b, rc);
    pv_ctx pc = {N, rc, c, rows, pl};
    run_parallel(nrows, 1, nthreads, pv_range, &pc);
    for (int64_t r = 0; r < nrows; ++r) p[r] = (double)pl[r];
    free(rc); free(pl);
    return ORACLE_OK;
}

/* ------------------------------------------- inverse: weights and constants */

/* Modified Chebyshev moments mu_n = int T_n(x) (1-x)^a (1+x)^b dx, n = 0..nmax,
 * by the forward three-term recurrence of Sec. 3.1 with the corrected mu_1. */
static void moments_l(int64_t nmax, real a, real b, real* mu)
{
    real lg = RLGAMMA(a + 1.0L) + RLGAMMA(b + 1.0L) - RLGAMMA(a + b + 2.0L);
    mu[0] = RPOW(2.0L, a + b + 1.0L) * REXP(lg);
    if (nmax >= 1) mu[1] = (b - a) / (a + b + 2.0L) * mu[0];
    for (int64_t n = 1; n < nmax; ++n) {
        real nn = (real)n;
        mu[n + 1] = -(2.0L * (a - b) * mu[n] + (a + b - nn + 2.0L) * mu[n - 1]) / (a + b + nn + 2.0L);
    }
}

int oracle_moments(int64_t nmax, double alpha, double beta, double* mu)
{
    if (nmax < 0 || !mu || !(alpha > -1.0) || !(beta > -1.0)) return ORACLE_EINVAL;
    real* m = (real*)malloc(sizeof(real) * (size_t)(nmax + 1));
    if (!m) return ORACLE_ENOMEM;
    moments_l(nmax, alpha, beta, m);
    for (int64_t n = 0; n <= nmax; ++n) mu[n] = (double)m[n];
    free(m);
    return ORACLE_OK;
}

typedef struct {
    int64_t L;          /* number of intervals: nodes j = 0..L */
    const real* mu;     /* mu_0..mu_L */
    const real* costab; /* cos(pi r / L), r = 0..2L-1 */
    real* w;
} ccw_ctx;

/* eq. CCweights: w_j = (1 - (d_j0 + d_jL)/2)/L {mu_0 + (-1)^j mu_L + 2 sum_{k=1}^{L-1} mu_k cos(pi k j / L)} */
static void ccw_range(int64_t lo, int64_t hi, void* vctx)
{
    ccw_ctx* x = (ccw_ctx*)vctx;
    int64_t L = x->L, P = 2 * L;
    for (int64_t j = lo; j < hi; ++j) {
        acc_t s = {0.0L, 0.0L};
        acc_add(&s, x->mu[0]);
        acc_add(&s, (j & 1) ? -x->mu[L] : x->mu[L]);
        int64_t r = j;
        for (int64_t k = 1; k < L; ++k) {
            acc_add(&s, 2.0L * x->mu[k] * x->costab[r]);
            r += j;
            if (r >= P) r -= P;
        }
        real wj = (j == 0 || j == L) ? 0.5L : 1.0L;
        x->w[j] = wj / (real)L * acc_get(&s);
    }
}

static int cc_weights_l(int64_t L, real a, real b, real* w, int nthreads)
{
    real* mu = (real*)malloc(sizeof(real) * (size_t)(L + 1));
    real* ct = (real*)malloc(sizeof(real) * (size_t)(2 * L));
    if (!mu || !ct) { free(mu); free(ct); return ORACLE_ENOMEM; }
    moments_l(L, a, b, mu);
    for (int64_t r = 0; r < 2 * L; ++r) ct[r] = cospi_frac(r, L);
    ccw_ctx cx = {L, mu, ct, w};
    run_parallel(L + 1, 64, nthreads, ccw_range, &cx);
    free(mu); free(ct);
    return ORACLE_OK;
}

/* Clenshaw--Curtis weights for the Jacobi weight on the L+1 points cos(pi j / L). */
int oracle_cc_weights(int64_t L, double alpha, double beta, double* w, int nthreads)
{
    if (L < 1 || !w || !(alpha > -1.0) || !(beta > -1.0)) return ORACLE_EINVAL;
    real* wl = (real*)malloc(sizeof(real) * (size_t)(L + 1));
    if (!wl) return ORACLE_ENOMEM;
    int st = cc_weights_l(L, alpha, beta, wl, nthreads);
    if (st == ORACLE_OK)
        for (int64_t j = 0; j <= L; ++j) w[j] = (double)wl[j];
    free(wl);
    return st;
}

/* Orthonormality constants of eq. Anab, n = 0..nmax.  A_0 and A_1 come from
 * the Gamma-function closed form; for n >= 2 the same closed form is advanced
 * by its exact ratio A_n / A_{n-1}, which avoids the cancellation of large
 * log-Gamma values. */
static void norm_consts_l(int64_t nmax, real a, real b, real* A)
{
    real two = RPOW(2.0L, a + b + 1.0L);
    A[0] = two * REXP(RLGAMMA(a + 1.0L) + RLGAMMA(b + 1.0L) - RLGAMMA(a + b + 2.0L));
    if (nmax >= 1)
        A[1] = two * REXP(RLGAMMA(a + 2.0L) + RLGAMMA(b + 2.0L) - RLGAMMA(a + b + 2.0L)) / (a + b + 3.0L);
    for (int64_t n = 2; n <= nmax; ++n) {
        real nn = (real)n;
        A[n] = A[n - 1] * (nn + a) * (nn + b) * (2.0L * nn + a + b - 1.0L) /
               ((2.0L * nn + a + b + 1.0L) * (nn + a + b) * nn);
    }
}

int oracle_norm_consts(int64_t nmax, double alpha, double beta, double* A)
{
    if (nmax < 0 || !A || !(alpha > -1.0) || !(beta > -1.0)) return ORACLE_EINVAL;
    real* al = (real*)malloc(sizeof(real) * (size_t)(nmax + 1));
    if (!al) return ORACLE_ENOMEM;
    norm_consts_l(nmax, alpha, beta, al);
    for (int64_t n = 0; n <= nmax; ++n) A[n] = (double)al[n];
    free(al);
    return ORACLE_OK;
}

/* ------------------------------------------------------------- inverse */

typedef struct {
    int64_t N;          /* coefficient degree; grid has 2N+1 points */
    const double* cheb;
    const real* costab; /* cos(pi r / (2N)), r = 0..4N-1 */
    real* f;
} fval_ctx;

/* f_j = sum_k c_k cos(pi j k / (2N)) = p_N(x_j) on the 2N+1 point grid. */
static void fval_range(int64_t lo, int64_t hi, void* vctx)
{
    fval_ctx* x = (fval_ctx*)vctx;
    int64_t N = x->N, P = 4 * N;
    for (int64_t j = lo; j < hi; ++j) {
        acc_t s = {0.0L, 0.0L};
        int64_t r = 0;
        for (int64_t k = 0; k <= N; ++k) {
            acc_add(&s, (real)x->cheb[k] * x->costab[r]);
            r += j;
            if (r >= P) r -= P;
        }
        x->f[j] = acc_get(&s);
    }
}

#define PROJ_BLOCKS 32

typedef struct {
    int64_t N;
    const rec_t* rc;
    const real* g;      /* w_j f_j on the 2N grid */
    real* part;         /* PROJ_BLOCKS x (N+1) sums */
    real* comp;         /* their compensation terms */
} proj_ctx;

/* Block of points -> partial y_n = sum_j P_n(x_j) g_j. */
static void proj_range(int64_t lo, int64_t hi, void* vctx)
{
    proj_ctx* x = (proj_ctx*)vctx;
    int64_t N = x->N, G = 2 * N;
    int64_t npts = G + 1;
    for (int64_t blk = lo; blk < hi; ++blk) {
        int64_t j0 = npts * blk / PROJ_BLOCKS, j1 = npts * (blk + 1) / PROJ_BLOCKS;
        real* s = x->part + (size_t)blk * (size_t)(N + 1);
        real* c = x->comp + (size_t)blk * (size_t)(N + 1);
        for (int64_t n = 0; n <= N; ++n) { s[n] = 0.0L; c[n] = 0.0L; }
        for (int64_t j = j0; j < j1; ++j) {
            real gj = x->g[j];
            if (gj == 0.0L) continue;
            walker_t w;
            walker_init(&w, j, G);
            for (int64_t n = 0; n <= N; ++n) {
                real v = w.p * gj;
                real t = s[n] + v;
                if (RFABS(s[n]) >= RFABS(v)) c[n] += (s[n] - t) + v;
                else c[n] += (v - t) + s[n];
                s[n] = t;
                if (n == N) break;
                walker_step(&w, x->rc, n);
            }
        }
    }
}

/* Inverse CJT: out[n], n = 0..N, from cheb[k], k = 0..N (eqs. iCJT, CJTT). */
int oracle_inverse(int64_t N, double alpha, double beta, const double* cheb, double* out, int nthreads)
{
    if (N < 1 || !cheb || !out) return ORACLE_EINVAL;
    if (!(alpha > -1.0) || !(beta > -1.0)) return ORACLE_EINVAL;
    real a = alpha, b = beta;
    int64_t G = 2 * N;
    real* ct = (real*)malloc(sizeof(real) * (size_t)(2 * G));
    real* f = (real*)malloc(sizeof(real) * (size_t)(G + 1));
    real* w = (real*)malloc(sizeof(real) * (size_t)(G + 1));
    rec_t* rc = (rec_t*)malloc(sizeof(rec_t) * (size_t)(N + 1));
    real* A = (real*)malloc(sizeof(real) * (size_t)(N + 1));
    real* part = (real*)malloc(sizeof(real) * (size_t)PROJ_BLOCKS * (size_t)(N + 1));
    real* comp = (real*)malloc(sizeof(real) * (size_t)PROJ_BLOCKS * (size_t)(N + 1));
    int st = ORACLE_OK;
    if (!ct || !f || !w || !rc || !A || !part || !comp) { st = ORACLE_ENOMEM; goto done; }

    for (int64_t r = 0; r < 2 * G; ++r) ct[r] = cospi_frac(r, G);
    {
        fval_ctx fc = {N, cheb, ct, f};
        run_parallel(G + 1, 64, nthreads, fval_range, &fc);
    }
    st = cc_weights_l(G, a, b, w, nthreads);
    if (st != ORACLE_OK) goto done;
    for (int64_t j = 0; j <= G; ++j) w[j] *= f[j];   /* g = w .* f */

    rec_coeffs(N, a, b, rc);
    {
        proj_ctx pc = {N, rc, w, part, comp};
        run_parallel(PROJ_BLOCKS, 1, nthreads, proj_range, &pc);
    }
    norm_consts_l(N, a, b, A);
    for (int64_t n = 0; n <= N; ++n) {
        acc_t s = {0.0L, 0.0L};
        for (int blk = 0; blk < PROJ_BLOCKS; ++blk) {
            acc_add(&s, part[(size_t)blk * (size_t)(N + 1) + (size_t)n]);
            acc_add(&s, comp[(size_t)blk * (size_t)(N + 1) + (size_t)n]);
        }
        out[n] = (double)(acc_get(&s) / A[n]);
    }
done:
    free(ct); free(f); free(w); free(rc); free(A); free(part); free(comp);
    return st;
}

/* Version tag of the oracle's arithmetic (bump when it changes). */
int oracle_version(void) { return 1; }
