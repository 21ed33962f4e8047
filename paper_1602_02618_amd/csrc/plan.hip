// Plan construction (Sec. 4, "Planification"): partition, recurrence
// coefficients, Hahn diagonals, Clenshaw--Curtis weights, orthonormality
// constants and recurrence work lists.  The partition and work lists are
// host-side integer bookkeeping over O(log N) window edges; every per-degree
// and per-point array is computed by a device kernel in FP64.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "cjt_internal.h"
#include "plan.h"
#include "planmath.h"

namespace cjt {

// ------------------------------------------------------------------ partition (Sec. 2.2)

namespace {

// log g_M(theta_i), theta_i = pi i / G: the envelope of |f_M| (Sec. 2.2),
// summed in log space; -inf when every coefficient vanishes (a = b = 1/2).
// log of the coefficients a_l b_{M-l} of g_M's terms (-inf for zero terms):
// independent of the angle, so computed once per (M, alpha, beta)
struct GmCoef {
    double lc[kMaxM + 2];
    int M;
};

GmCoef gm_coef(int M, const double* ca, const double* cb)
{
    GmCoef g;
    g.M = M;
    for (int l = 0; l <= M; ++l) {
        const double coef = ca[l] * cb[M - l];
        g.lc[l] = coef > 0.0 ? log(coef) : -INFINITY;
    }
    return g;
}

double log_gM(double th2, const GmCoef& g, double a, double b)
{
    const int M = g.M;
    const double ls = log(sin(th2)), lc = log(cos(th2));
    double t[kMaxM + 2];
    int nt = 0;
    double mx = -INFINITY;
    for (int l = 0; l <= M; ++l) {
        if (g.lc[l] == -INFINITY) continue;
        t[nt] = g.lc[l] + (l - M - b - 0.5) * lc - (l + a + 0.5) * ls;
        mx = fmax(mx, t[nt]);
        ++nt;
    }
    if (nt == 0) return -INFINITY;
    double s = 0.0;
    for (int q = 0; q < nt; ++q) s += exp(t[q] - mx);
    return mx + log(s);
}


}  // namespace

void compute_partition(int64_t G, int64_t cap, double a, double b, int M, Part* P)
{
    *P = Part{};
    P->G = G;
    P->cap = cap;
    P->M = M;
    double ca[kMaxM + 2], cb[kMaxM + 2];
    hahn_pochhammer(M, a, b, ca, cb);
    const GmCoef gc = gm_coef(M, ca, cb);
    auto lg = [&](int64_t i) { return log_gM(kPi * (double)i / (2.0 * (double)G), gc, a, b); };
    const double leps = log(kEps);
    const double lg_half = log_gM(kPi / 4.0, gc, a, b);  // g_M(pi/2)
    const int64_t ncap1 = cap + 1;
    P->rec_entries = (G + 1) * ncap1;
    if (lg_half == -INFINITY) {
        // f_m = 0 for m >= 1: Hahn's expansion with one term is exact (a = b = 1/2).
        P->exact = 1;
        P->M = 1;
        P->n_M = 1;
        P->alpha_N = 0.5;
        P->K = 1;
        P->theta_bar = G / 2;
        if (G >= 2 && cap >= 2) {
            P->nblk = 1;
            P->deg_lo[0] = 2;
            P->deg_hi[0] = ncap1;
            P->win_lo[0] = 1;
            P->win_hi[0] = G - 1;
            P->rec_entries -= (G - 1) * (ncap1 - 2);
        }
        return;
    }
    // n_M = floor((eps 2^(2M-1) sqrt(pi) / g_M(pi/2))^(-1/(M+1/2)))
    const double lnM = -(leps + (2.0 * M - 1.0) * log(2.0) + 0.5 * log(kPi) - lg_half) / (M + 0.5);
    P->n_M = lnM > 60.0 ? ((int64_t)1 << 60) : (int64_t)floor(exp(lnM));
    if (P->n_M < 1) P->n_M = 1;
    if (G < 3 || G <= P->n_M) return;
    P->alpha_N = fmin(1.0 / log((double)G / (double)P->n_M), 0.5);
    P->K = (int)ceil(log((double)G / (double)P->n_M) / log(1.0 / P->alpha_N));
    // discrete minimiser of g_M over i = 1..G-1 (g_M is convex on (0, pi):
    // each term is a positive multiple of sin^-p(theta/2) cos^-q(theta/2), p, q > 0)
    int64_t lo = 1, hi = G - 1;
    while (lo < hi) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (lg(mid + 1) >= lg(mid)) hi = mid;
        else lo = mid + 1;
    }
    const int64_t tb = lo;
    P->theta_bar = tb;
    const double lgb = lg(tb);
    int64_t prev_cut = ncap1;
    for (int k = 1; k <= kMaxBlocks; ++k) {
        const int64_t jk = (int64_t)floor(pow(P->alpha_N, k) * (double)G);
        if (jk <= P->n_M || jk < 2) break;
        const double l2c = log(2.0) + hahn_logC((double)jk, P->M, a, b);
        if (!(l2c + lgb < leps)) break;
        // contiguous window around theta_bar where 2 C_{jk,M} g_M < eps
        int64_t L = 1, R = tb;
        while (L < R) {
            const int64_t mid = L + (R - L) / 2;
            if (l2c + lg(mid) < leps) R = mid;
            else L = mid + 1;
        }
        const int64_t wlo = L;
        L = tb;
        R = G - 1;
        while (L < R) {
            const int64_t mid = L + (R - L + 1) / 2;
            if (l2c + lg(mid) < leps) L = mid;
            else R = mid - 1;
        }
        const int64_t whi = L;
        const int64_t dlo = std::min(jk, ncap1);
        const int64_t dhi = prev_cut;
        if (dlo < dhi) {
            const int q = P->nblk++;
            P->deg_lo[q] = dlo;
            P->deg_hi[q] = dhi;
            P->win_lo[q] = wlo;
            P->win_hi[q] = whi;
            P->rec_entries -= (whi - wlo + 1) * (dhi - dlo);
        }
        prev_cut = std::min(prev_cut, dlo);
    }
}

// cut(i): degrees [0, cut) of grid point i left to recurrence.
static int64_t point_cut(const Part& P, int64_t i)
{
    int64_t c = P.cap + 1;
    for (int k = 0; k < P.nblk; ++k)
        if (i >= P.win_lo[k] && i <= P.win_hi[k]) c = P.deg_lo[k];
    return c;
}

// Switch rule (Sec. 4.2): modified recurrences for theta <= pi/4 and >= 3pi/4.
static int point_mode(int64_t i, int64_t G)
{
    if (4 * i <= G) return +1;
    if (4 * i >= 3 * G) return -1;
    return 0;
}

void build_tasks(const Part& P, int width, std::vector<RecTask>* out, int64_t* part_total)
{
    const int64_t G = P.G;
    std::vector<int64_t> bp = {0, G + 1, G / 4 + 1, (3 * G + 3) / 4};
    for (int k = 0; k < P.nblk; ++k) {
        bp.push_back(P.win_lo[k]);
        bp.push_back(P.win_hi[k] + 1);
    }
    std::sort(bp.begin(), bp.end());
    bp.erase(std::unique(bp.begin(), bp.end()), bp.end());
    out->clear();
    for (size_t s = 0; s + 1 < bp.size(); ++s) {
        int64_t a = bp[s], e = bp[s + 1];
        if (a < 0) a = 0;
        if (e > G + 1) e = G + 1;
        if (a >= e) continue;
        const int64_t cut = point_cut(P, a);
        const int mode = point_mode(a, G);
        for (int64_t p = a; p < e; p += width) {
            RecTask t;
            t.p0 = (int32_t)p;
            t.np = (int32_t)std::min<int64_t>(width, e - p);
            t.mode = mode;
            t.cut = (int32_t)cut;
            t.off = 0;
            out->push_back(t);
        }
    }
    std::stable_sort(out->begin(), out->end(), [](const RecTask& x, const RecTask& y) { return x.cut > y.cut; });
    int64_t off = 0;
    for (auto& t : *out) {
        t.off = off;
        off += t.cut;
    }
    *part_total = off;
}

// ------------------------------------------------------------------ M selection

// Predicted GPU cost of one forward plus one inverse transform for a given M:
// Hahn blocks cost one complex FFT of length L per (block, term), counted as
// 5 L log2 L, and the recurrence a weight per (point, degree) pair.  The
// weight is calibrated on MI355X step times of batched transforms: one
// pair costs about as much as one FFT "flop" (the FFT passes move their
// intermediates through memory while the recurrences run from registers on a
// concurrent stream), which puts the optimum at M = 7-8 for N up to 2e5.  Very
// large degrees usually run in small batches, where the recurrences' serial
// chains are exposed; above N = 2^18 their weight grows to 3.5 at N = 2^20.
static double plan_cost(int64_t N, const Part& f, const Part& i)
{
    auto fft = [](double L) { return 5.0 * L * log2(fmax(L, 2.0)); };
    const double big = log2((double)N / 262144.0);
    const double rec = big > 0.0 ? 1.0 + 1.25 * big : 1.0;
    return f.nblk * f.M * fft((double)N) + i.nblk * i.M * fft(2.0 * (double)N) +
           rec * (double)(f.rec_entries + i.rec_entries);
}

void choose_partitions(int64_t N, double a, double b, int M, Part* f, Part* inv)
{
    if (M > 0) {
        compute_partition(N, N, a, b, M, f);
        compute_partition(2 * N, N, a, b, M, inv);
        return;
    }
    // the model falls with M (fewer recurrence entries) until the Hahn-block
    // transforms dominate and then rises; the sweep stops three terms past the
    // last improvement (the first minimiser, as in a full sweep over 5..20)
    double best = INFINITY;
    int since = 0;
    for (int m = 5; m <= 20 && since < 3; ++m) {
        Part pf, pi;
        compute_partition(N, N, a, b, m, &pf);
        compute_partition(2 * N, N, a, b, m, &pi);
        const double c = plan_cost(N, pf, pi);
        if (c < best) {
            best = c;
            *f = pf;
            *inv = pi;
            since = 0;
        } else {
            ++since;
        }
    }
}

// ------------------------------------------------------------------ device kernels

// Recurrence coefficients (Sec. 1.2) and the endpoint ratios of Sec. 4.2.
//   f0[n] = (A_n, B_n, C_{n+1})                    forward, three-term
//   fp/fm[n] = (A_n, C_{n+1} rb_{n+1}, 1/rb_n)     forward, modified at x0 = +1 / -1
//   i0[n] = (A_n, B_n, C_n)                        inverse, three-term
//   ip/im[n] = (A_n, C_n / rf_{n-1}, rf_n)         inverse, modified at x0 = +1 / -1
__device__ inline void rec_ABC(double n, double a, double b, double* A, double* B, double* C)
{
    if (n == 0.0) {
        *A = 0.5 * (a + b + 2.0);
        *B = 0.5 * (a - b);
        *C = 0.0;
        return;
    }
    const double s = 2.0 * n + a + b;
    const double den = 2.0 * (n + 1.0) * (n + a + b + 1.0);
    *A = (s + 1.0) * (s + 2.0) / den;
    *B = (a - b) * (a + b) * (s + 1.0) / (den * s);
    *C = (n + a) * (n + b) * (s + 2.0) / ((n + 1.0) * (n + a + b + 1.0) * s);
}

// r^b_n(+-1) of the lemma in Sec. 4.2, n >= 1.
__device__ inline double rb_pm(double n, double a, double b, int side)
{
    const double r = (n + 1.0) / n * (a + b + n + 1.0) * (a + b + 2.0 * n) / ((a + b + 2.0 * n + 2.0));
    return side > 0 ? r / (n + b) : -r / (n + a);
}

// r^f_n(+-1) = P_{n+1}(+-1) / P_n(+-1) (Sec. 4.2).
__device__ inline double rf_pm(double n, double a, double b, int side)
{
    return side > 0 ? (n + a + 1.0) / (n + 1.0) : -(n + b + 1.0) / (n + 1.0);
}

__global__ void k_plan_rec(int64_t N, double a, double b, d4* f0, d4* fp, d4* fm, d4* i0,
                           d4* ip, d4* im)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n > N) return;
    const double dn = (double)n;
    double A, B, C, A1, B1, C1;
    rec_ABC(dn, a, b, &A, &B, &C);
    rec_ABC(dn + 1.0, a, b, &A1, &B1, &C1);
    f0[n] = d4{A, B, C1, 0.0};
    i0[n] = d4{A, B, C, 0.0};
    const double rbp1 = rb_pm(dn + 1.0, a, b, +1), rbm1 = rb_pm(dn + 1.0, a, b, -1);
    const double rbip = n >= 1 ? 1.0 / rb_pm(dn, a, b, +1) : 0.0;
    const double rbim = n >= 1 ? 1.0 / rb_pm(dn, a, b, -1) : 0.0;
    fp[n] = d4{A, C1 * rbp1, rbip, 0.0};
    fm[n] = d4{A, C1 * rbm1, rbim, 0.0};
    const double hp = n >= 1 ? C / rf_pm(dn - 1.0, a, b, +1) : 0.0;
    const double hm = n >= 1 ? C / rf_pm(dn - 1.0, a, b, -1) : 0.0;
    ip[n] = d4{A, hp, rf_pm(dn, a, b, +1), 0.0};
    im[n] = d4{A, hm, rf_pm(dn, a, b, -1), 0.0};
}

// C_{n,m}, m < M, for n >= nlo (zero below): eq. Cnmabasy at m = 0, then the
// m-step of eq. Cnmabrec.
// Power-of-two exponents e_m of the Hahn terms: C_{n,m} is stored times 2^e_m
// and (u_m, v_m) times 2^-e_m, so every product C_{n,m} (u_m, v_m) is
// unchanged exactly while the inputs of FP32 block transforms (C_{n,m} c_n,
// or (u_m, v_m) g) stay inside the FP32 exponent range.  Zero for FP64 plans.
struct TermScale {
    int e[kMaxM];
};

__global__ void k_plan_C(int64_t N, double a, double b, int M, int64_t nlo, TermScale ts, double* C)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n > N) return;
    if (n < nlo) {
        for (int m = 0; m < M; ++m) C[(int64_t)m * (N + 1) + n] = 0.0;
        return;
    }
    const double dn = (double)n;
    double c = hahn_C(dn, 0, a, b);
    C[n] = ldexp(c, ts.e[0]);
    for (int m = 1; m < M; ++m) {
        c /= 2.0 * (2.0 * dn + a + b + m + 1.0);
        C[(int64_t)m * (N + 1) + n] = ldexp(c, ts.e[m]);
    }
}

// (u_m, v_m)(theta_i), theta_i = pi i / G, on [lo, hi] (zero elsewhere), from
//   u_m + i v_m = sum_l a_l b_{m-l} exp(i theta_{m,l}) / (sin^{l+a+1/2}(theta/2) cos^{m-l+b+1/2}(theta/2))
// with theta_{m,l} = (a + l + 1/2) pi/2 - (a + b + m + 1) theta/2 (Sec. 2.1, eq. Jacasyuv):
// = K c^-m e^{i phi_0} e^{-i m theta/2} sum_l a_l b_{m-l} (i t)^l,
//   t = cot(theta/2), K = s^-(a+1/2) c^-(b+1/2), phi_0 = (a+1/2) pi/2 - (a+b+1) theta/2.
//
// The forward blocks take (u_m, v_m) interleaved.  The transposed blocks of
// the inverse (halves = true) take, per term, the two planes
// S = (u_m + v_m)/2 and D = (u_m - v_m)/2 of G+1 values each, stored back to
// back in the same G+1 complex slots: the real-input FFT's r is then one
// product per element, r_j = S_j g_j and r_{2G-j} = D_j g_j.
__device__ __forceinline__ void put_uv(cx<double>* uv, int64_t G, int m, int64_t i, double u, double v, bool halves)
{
    if (!halves) {
        uv[(int64_t)m * (G + 1) + i] = {u, v};
        return;
    }
    double* S = reinterpret_cast<double*>(uv + (int64_t)m * (G + 1));
    S[i] = 0.5 * (u + v);
    S[G + 1 + i] = 0.5 * (u - v);
}

__global__ void k_plan_uv(int64_t G, double a, double b, int M, int64_t lo, int64_t hi, TermScale ts,
                          cx<double>* uv, bool halves)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i > G) return;
    if (i < lo || i > hi || i <= 0 || i >= G) {
        for (int m = 0; m < M; ++m) put_uv(uv, G, m, i, 0.0, 0.0, halves);
        return;
    }
    double ca[kMaxM + 1], cb[kMaxM + 1];
    hahn_pochhammer(M, a, b, ca, cb);
    double s, c;
    sincospi((double)i / (double)(2 * G), &s, &c);
    const double t = c / s;
    const double K = exp(-(a + 0.5) * log(s) - (b + 0.5) * log(c));
    double e0s, e0c;
    sincospi(0.5 * (a + 0.5) - (a + b + 1.0) * (double)i / (double)(2 * G), &e0s, &e0c);
    double tp[kMaxM + 1];
    tp[0] = 1.0;
    for (int l = 1; l < M; ++l) tp[l] = tp[l - 1] * t;
    double cm = K;  // K c^-m
    const double ic = 1.0 / c;
    const int64_t fourG = 4 * G;
    for (int m = 0; m < M; ++m) {
        double wr = 0.0, wi = 0.0;
        for (int l = 0; l <= m; ++l) {
            const double term = ca[l] * cb[m - l] * tp[l];
            switch (l & 3) {
                case 0: wr += term; break;
                case 1: wi += term; break;
                case 2: wr -= term; break;
                default: wi -= term; break;
            }
        }
        // e^{-i pi m i / (2G)} from the exact rational angle
        const int64_t r = ((int64_t)m * i) % fourG;
        double rs, rc;
        sincospi((double)r / (double)(2 * G), &rs, &rc);
        // e^{i phi_0} e^{-i m theta/2}
        const double er = e0c * rc + e0s * rs;
        const double ei = e0s * rc - e0c * rs;
        const double vr = cm * (er * wr - ei * wi);
        const double vi = cm * (er * wi + ei * wr);
        put_uv(uv, G, m, i, ldexp(vr, -ts.e[m]), ldexp(vi, -ts.e[m]), halves);
        cm *= ic;
    }
}

// s_n = 1 / A_n (eq. Anab via eq. Anabasy).
__global__ void k_plan_s(int64_t N, double a, double b, double* s)
{
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n > N) return;
    s[n] = 1.0 / jacobi_norm((double)n, a, b);
}

// ------------------------------------------------------------------ host plan build

// Modified Chebyshev moments of the Jacobi weight (Sec. 3.1): mu_0 from the
// Beta function, mu_1 = (b - a)/(a + b + 2) mu_0 (integration by parts; the
// printed (a - b) has the wrong sign), then the forward three-term recurrence.
static void moments_host(int64_t L, double a, double b, std::vector<double>* mu)
{
    mu->assign(L + 1, 0.0);
    (*mu)[0] = exp2(a + b + 1.0) * tgamma(a + 1.0) * tgamma(b + 1.0) / tgamma(a + b + 2.0);
    if (L >= 1) (*mu)[1] = (b - a) / (a + b + 2.0) * (*mu)[0];
    for (int64_t n = 1; n < L; ++n) {
        const double dn = (double)n;
        (*mu)[n + 1] = -(2.0 * (a - b) * (*mu)[n] + (a + b - dn + 2.0) * (*mu)[n - 1]) / (a + b + dn + 2.0);
    }
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

namespace {

// log2 of a bound of |u_m + i v_m| at theta (the sum of the absolute values of
// the terms of eq. Jacasyuv).
double log2_uv_bound(double theta, int m, double a, double b, const double* ca, const double* cb)
{
    const double s = sin(0.5 * theta), c = cos(0.5 * theta), t = c / s;
    double sum = 0.0, tp = 1.0;
    for (int l = 0; l <= m; ++l) {
        sum += fabs(ca[l] * cb[m - l]) * tp;
        tp *= t;
    }
    return (-(a + 0.5) * log(s) - (b + 0.5 + m) * log(c) + log(sum)) / log(2.0);
}

// Term exponents of an FP32-bulk plan: e_m scales the largest (u_m, v_m) on
// the block-0 windows of both grids (the widest windows) to about 1; then
// C_{n,m} 2^e_m is at most about the Hahn term bound on those windows, which
// is below 1 there.  FP64 plans keep e_m = 0.
TermScale term_scale(const Plan& P)
{
    TermScale ts{};
    if (!(P.flags & CJT_FP32_BULK)) return ts;
    const int M = std::max(P.fwd.M, P.inv.M);
    double ca[kMaxM + 1], cb[kMaxM + 1];
    hahn_pochhammer(M, P.alpha, P.beta, ca, cb);
    for (int m = 0; m < M; ++m) {
        double e = 0.0;
        bool any = false;
        for (const Part* pt : {&P.fwd, &P.inv}) {
            if (pt->nblk == 0) continue;
            for (int64_t i : {pt->win_lo[0], pt->win_hi[0]}) {
                if (i <= 0 || i >= pt->G) continue;
                const double l2 = log2_uv_bound(kPi * (double)i / (double)pt->G, m, P.alpha, P.beta, ca, cb);
                e = any ? std::max(e, l2) : l2;
                any = true;
            }
        }
        ts.e[m] = any ? (int)std::min(std::max(floor(e), -900.0), 900.0) : 0;
    }
    return ts;
}

// Byte offsets of a plan's device arrays in its arena.
struct Layout {
    size_t C, UVf, UVi, W, S, R, Tf, Ti, Mu, Gf, Gi, Gbf, Gbi, total;
};

Layout layout_of(const Plan& P)
{
    const int64_t N = P.N, nf = N + 1, ni = 2 * N + 1;
    const int M = std::max(P.fwd.M, P.inv.M);
    const bool fp32 = (P.flags & CJT_FP32_BULK) != 0;
    Layout l{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return o;
    };
    l.C = take(sizeof(double) * (size_t)M * nf);
    l.UVf = take(sizeof(cx<double>) * (size_t)P.fwd.M * nf);
    l.UVi = take(sizeof(cx<double>) * (size_t)P.inv.M * ni);
    l.W = take(sizeof(double) * ni);
    l.S = take(sizeof(double) * nf);
    l.R = take(sizeof(d4) * 6 * (size_t)nf);
    l.Tf = take(sizeof(RecTask) * std::max<size_t>(1, P.tasks_f.size()));
    l.Ti = take(sizeof(RecTask) * std::max<size_t>(1, P.tasks_i.size()));
    l.Mu = take(sizeof(double) * ni);
    FftGeom gf, gi;
    geometry_shape(N, &gf, P.lg1_f);
    geometry_shape(2 * N, &gi, P.lg1_i);
    l.Gf = take(gf.bluestein ? chirp_table_bytes(gf, false) : 0);
    l.Gi = take(gi.bluestein ? chirp_table_bytes(gi, false) : 0);
    l.Gbf = take(fp32 && gf.bluestein ? chirp_table_bytes(gf, true) : 0);
    l.Gbi = take(fp32 && gi.bluestein ? chirp_table_bytes(gi, true) : 0);
    l.total = off;
    return l;
}

// The Clenshaw--Curtis weights program: one DCT-I of the moments on the 2N grid.
cjt_status weights_program(const Plan& P, const FftGeom& gi, Program* pr)
{
    ExecDesc d{};
    d.N = P.N;
    d.G = 2 * P.N;
    d.alpha = P.alpha;
    d.beta = P.beta;
    d.geo = gi;
    d.geob = gi;
    pr->descs.push_back(d);
    std::vector<double> fl(1, 0.0), by(1, 0.0);
    return add_fft(*pr, std::vector<int>{0}, Src::Moments, Sink::Weights, false, 0, nullptr, nullptr, fl, by);
}

}  // namespace

int64_t fft_power_length(int64_t L)
{
    FftGeom g;
    geometry_shape(L, &g, -1);
    return g.bluestein ? g.P : g.L;
}

void plan_layout(Plan* P)
{
    // two-pass splits from the schedule table (the library default where untuned)
    const bool fp32 = (P->flags & CJT_FP32_BULK) != 0;
    {
        FftGeom g;
        geometry_shape(P->N, &g, -1);
        P->lg1_f = tuned_split(fft_power_length(P->N), fp32, g.bluestein != 0, false);
        geometry_shape(2 * P->N, &g, -1);
        P->lg1_i = tuned_split(fft_power_length(2 * P->N), fp32, g.bluestein != 0, true);
    }
    const Layout l = layout_of(*P);
    P->arena_bytes = l.total;
    FftGeom gf, gi;
    geometry_shape(P->N, &gf, P->lg1_f);
    geometry_shape(2 * P->N, &gi, P->lg1_i);
    size_t scr = 0;
    for (const FftGeom* g : {&gf, &gi})
        if (g->bluestein) scr = std::max(scr, chirp_scratch_bytes(*g, fp32));
    Program pr;
    size_t items = 1;
    if (weights_program(*P, gi, &pr) == CJT_OK) items = std::max<size_t>(1, pr.items.size());
    const size_t wprog = align_up(sizeof(ExecDesc)) + align_up(sizeof(Item) * items) + fft_job_bytes(2 * P->N, false);
    P->scratch_bytes = std::max(scr, wprog);
}

cjt_status build_plan_device(Plan* P, hipStream_t st, void* arena, void* scratch)
{
    const int64_t N = P->N;
    const int M = std::max(P->fwd.M, P->inv.M);
    const int64_t nf = N + 1, ni = 2 * N + 1;
    const bool fp32 = (P->flags & CJT_FP32_BULK) != 0;
    const Layout ly = layout_of(*P);
    P->arena_bytes = ly.total;
    if (!arena) {
        CJT_HIP_TRY(hipMalloc(&arena, ly.total));
        P->own_arena = true;
    }
    P->arena = arena;
    char* scr = (char*)scratch;
    if (!scr && hipMalloc((void**)&scr, std::max<size_t>(P->scratch_bytes, 256)) != hipSuccess)
        return fail(CJT_ENOMEM, "plan scratch allocation failed");
    char* base = (char*)arena;
    P->C = (double*)(base + ly.C);
    P->uv_f = (cx<double>*)(base + ly.UVf);
    P->uv_i = (cx<double>*)(base + ly.UVi);
    P->w = (double*)(base + ly.W);
    P->s = (double*)(base + ly.S);
    d4* R = (d4*)(base + ly.R);
    P->f0 = R;
    P->fp = R + nf;
    P->fm = R + 2 * nf;
    P->i0 = R + 3 * nf;
    P->ip = R + 4 * nf;
    P->im = R + 5 * nf;
    P->d_tasks_f = (RecTask*)(base + ly.Tf);
    P->d_tasks_i = (RecTask*)(base + ly.Ti);
    double* mu = (double*)(base + ly.Mu);

    cjt_status stt = CJT_OK;
    std::vector<double> hmu;
    do {
        // FFT geometries of both grids; chirp-z tables live in the arena
        if ((stt = fft_geometry(N, false, st, &P->geo_f, base + ly.Gf, scr, P->lg1_f)) != CJT_OK) break;
        if ((stt = fft_geometry(2 * N, false, st, &P->geo_i, base + ly.Gi, scr, P->lg1_i)) != CJT_OK) break;
        P->geob_f = P->geo_f;
        P->geob_i = P->geo_i;
        if (fp32) {
            if ((stt = fft_geometry(N, true, st, &P->geob_f, base + ly.Gbf, scr, P->lg1_f)) != CJT_OK) break;
            if ((stt = fft_geometry(2 * N, true, st, &P->geob_i, base + ly.Gbi, scr, P->lg1_i)) != CJT_OK) break;
        }
        const double a = P->alpha, b = P->beta;
        const unsigned bs = 256;
        auto grid = [&](int64_t n) { return dim3((unsigned)((n + bs - 1) / bs)); };
        hipLaunchKernelGGL(k_plan_rec, grid(nf), dim3(bs), 0, st, N, a, b, P->f0, P->fp, P->fm, P->i0, P->ip,
                           P->im);
        int64_t nlo = N + 1;
        for (int k = 0; k < P->fwd.nblk; ++k) nlo = std::min(nlo, P->fwd.deg_lo[k]);
        for (int k = 0; k < P->inv.nblk; ++k) nlo = std::min(nlo, P->inv.deg_lo[k]);
        const TermScale ts = term_scale(*P);
        hipLaunchKernelGGL(k_plan_C, grid(nf), dim3(bs), 0, st, N, a, b, M, nlo, ts, P->C);
        const int64_t flo = P->fwd.nblk ? P->fwd.win_lo[0] : 1, fhi = P->fwd.nblk ? P->fwd.win_hi[0] : 0;
        hipLaunchKernelGGL(k_plan_uv, grid(nf), dim3(bs), 0, st, N, a, b, P->fwd.M, flo, fhi, ts, P->uv_f, false);
        const int64_t ilo = P->inv.nblk ? P->inv.win_lo[0] : 1, ihi = P->inv.nblk ? P->inv.win_hi[0] : 0;
        hipLaunchKernelGGL(k_plan_uv, grid(ni), dim3(bs), 0, st, 2 * N, a, b, P->inv.M, ilo, ihi, ts, P->uv_i, true);
        hipLaunchKernelGGL(k_plan_s, grid(nf), dim3(bs), 0, st, N, a, b, P->s);
        if (hipGetLastError() != hipSuccess) {
            stt = fail(CJT_EDEVICE, "plan kernel launch failed");
            break;
        }
        if ((!P->tasks_f.empty() &&
             hipMemcpyAsync(P->d_tasks_f, P->tasks_f.data(), sizeof(RecTask) * P->tasks_f.size(),
                            hipMemcpyHostToDevice, st) != hipSuccess) ||
            (!P->tasks_i.empty() &&
             hipMemcpyAsync(P->d_tasks_i, P->tasks_i.data(), sizeof(RecTask) * P->tasks_i.size(),
                            hipMemcpyHostToDevice, st) != hipSuccess)) {
            stt = fail(CJT_EDEVICE, "task copy failed");
            break;
        }
        moments_host(2 * N, a, b, &hmu);
        if (hipMemcpyAsync(mu, hmu.data(), sizeof(double) * ni, hipMemcpyHostToDevice, st) != hipSuccess) {
            stt = fail(CJT_EDEVICE, "moment copy failed");
            break;
        }
        // Clenshaw--Curtis weights on the 2N grid: one DCT-I of the moments
        // (scratch: [descriptor | items | FFT intermediates]).
        Program pr;
        if ((stt = weights_program(*P, P->geo_i, &pr)) != CJT_OK) break;
        const size_t dbytes = align_up(sizeof(ExecDesc));
        const size_t ibytes = align_up(sizeof(Item) * pr.items.size());
        pr.descs[0].in = mu;
        pr.descs[0].out = P->w;
        pr.descs[0].tmp = fft_job_bytes(2 * N, false) ? (void*)(scr + dbytes + ibytes) : nullptr;
        if (dbytes + ibytes + fft_job_bytes(2 * N, false) > std::max<size_t>(P->scratch_bytes, 256)) {
            stt = fail(CJT_EINVAL, "plan scratch too small");
            break;
        }
        if (hipMemcpyAsync(scr, pr.descs.data(), sizeof(ExecDesc), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(scr + dbytes, pr.items.data(), sizeof(Item) * pr.items.size(), hipMemcpyHostToDevice,
                           st) != hipSuccess) {
            stt = fail(CJT_EDEVICE, "descriptor copy failed");
            break;
        }
        for (const Launch& L : pr.launches) {
            stt = launch_fft(L, (const ExecDesc*)scr, (const Item*)(scr + dbytes) + L.item_off, st);
            if (stt != CJT_OK) break;
        }
    } while (0);
    if (hipStreamSynchronize(st) != hipSuccess && stt == CJT_OK) stt = fail(CJT_EDEVICE, "plan build failed");
    if (!scratch) (void)hipFree(scr);
    if (stt != CJT_OK && P->own_arena) {
        (void)hipFree(P->arena);
        P->arena = nullptr;
        P->own_arena = false;
    }
    return stt;
}

// ------------------------------------------------------------------ FFT geometry

namespace {
std::mutex g_tw_mu;
struct TwEntry {
    int dev;
    int64_t F;
    bool fp32;
    const void* tw;
};
std::vector<TwEntry> g_tw;  // power-of-two twiddle tables, one per (device, length, precision)

int ilog2_ceil(int64_t x)
{
    int lg = 0;
    while (((int64_t)1 << lg) < x) ++lg;
    return lg;
}

void split(FftGeom* g, int lg, int64_t F, int lg1)
{
    g->single = F <= kSingleMax ? 1 : 0;
    if (!g->single) {
        int lo = 0, hi = 0;
        split_range(lg, &lo, &hi);
        g->logL1 = lg1 >= lo && lg1 <= hi ? lg1 : lg / 2;
        g->logL2 = lg - g->logL1;
        g->L1 = 1 << g->logL1;
        g->L2 = 1 << g->logL2;
    }
}
}  // namespace

// Column lengths 2^lg1 the two-pass kernels accept for a length 2^lg: at
// least 16 and at most 2048 points on either side (16 values per thread, at
// most 2048 points per workgroup pass).
void split_range(int lg, int* lo, int* hi)
{
    *lo = std::max(4, lg - 11);
    *hi = std::min(11, lg - 4);
}

// Twiddles e^{i pi q / F}, q < 2F, of a power-of-two length F, built once per
// (device, F, precision) and kept for the life of the process (at most one
// table per power of two: 2F complex values each).
cjt_status fft_twiddles_cached(int64_t F, bool fp32, hipStream_t st, const void** out)
{
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_tw_mu);
    for (const TwEntry& e : g_tw)
        if (e.dev == dev && e.F == F && e.fp32 == fp32) {
            *out = e.tw;
            return CJT_OK;
        }
    const void* tw = nullptr;
    cjt_status s = make_twiddles(F, fp32, &tw, st);
    if (s != CJT_OK) return s;
    CJT_HIP_TRY(hipStreamSynchronize(st));
    g_tw.push_back(TwEntry{dev, F, fp32, tw});
    *out = tw;
    return CJT_OK;
}

// Shape of the length-L complex FFT: power-of-two lengths run directly (one
// or two passes), every other length through the chirp-z convolution of
// power-of-two length P >= 2L - 1.
void geometry_shape(int64_t L, FftGeom* g, int lg1)
{
    *g = FftGeom{};
    g->L = L;
    g->logL = ilog2_ceil(L);
    if ((L & (L - 1)) == 0) {
        split(g, g->logL, L, lg1);
    } else {
        g->bluestein = 1;
        g->logP = ilog2_ceil(2 * L - 1);
        g->P = (int64_t)1 << g->logP;
        split(g, g->logP, g->P, lg1);
    }
}

cjt_status fft_geometry(int64_t L, bool fp32, hipStream_t st, FftGeom* g, char* mem, char* scratch, int lg1)
{
    if (L < 1) return fail(CJT_EINVAL, "FFT length must be positive");
    geometry_shape(L, g, lg1);
    const int64_t F = g->bluestein ? g->P : L;
    cjt_status s = fft_twiddles_cached(F, fp32, st, &g->tw);
    if (s != CJT_OK) return s;
    if (!g->single) {
        if ((s = fft_twiddles_cached(g->L1, fp32, st, &g->tw1)) != CJT_OK) return s;
        if ((s = fft_twiddles_cached(g->L2, fp32, st, &g->tw2)) != CJT_OK) return s;
    }
    if (g->bluestein) {
        if (!mem || !scratch) return fail(CJT_EINVAL, "chirp-z tables need plan memory");
        s = make_chirp_tables(g, fp32, st, mem, scratch);
    }
    return s;
}

}  // namespace cjt
