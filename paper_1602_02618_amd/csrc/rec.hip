// Recurrence part of the transform: the entries of P_N (forward) and of its
// transpose (inverse) that lie outside every Hahn block (Sec. 2.2, P^REC).
//
// Forward: p_i = sum_{n < cut(i)} c_n P_n(x_i) by the Clenshaw--Smith algorithm
// (Sec. 4.2, Algorithm with u_{N+1} = u_{N+2} = 0), or, for theta_i <= pi/4 and
// >= 3pi/4, by its Reinsch-modified form anchored at x0 = +1 / -1 (Sec. 4.2)
// with the ratios r^b_n(+-1) of the lemma there.  With D_n = d_n / r^b_n the
// modified algorithm reads
//     D_n = A_n (x - x0) u_{n+1} + C_{n+1} r^b_{n+1} D_{n+1} + c_n,
//     u_n = u_{n+1} / r^b_n + D_n,
// and its final step A_0 (x - x0) u_1 + C_1 d_1 + c_0 is the same formula at
// n = 0, so p = D_0.  x - 1 = -2 sin^2(theta/2), x + 1 = 2 cos^2(theta/2).
//
// Inverse: y_n = sum_j P_n(x_j) g_j over the points j of the 2N grid whose
// recurrence range covers n (Sec. 3.2).  P_n(x_j) g_j comes from the
// three-term recurrence started at P_0 = g_j (linearity), or near the ends
// from the modified forward recurrence of Sec. 4.2 with r^f_n(+-1); with
// e_{n+1} = d_{n+1} r^f_n it reads
//     e_{n+1} = A_n (x - x0) pi_n + (C_n / r^f_{n-1}) e_n,   pi_{n+1} = r^f_n pi_n + e_{n+1}.
// Each thread carries kPPT points; per 16 degrees the wave sums its 64*kPPT
// values per degree through LDS and writes one partial sum per task and
// degree; a second kernel adds the partials of all tasks in a fixed order.
//
// Evaluation points.  P_n(cos theta) oscillates with frequency n in theta, so a
// point rounded to FP64 (relative error eps in theta or in x -+ 1) shifts
// P_n by about eps n theta, the same sign for every degree: near the ends,
// where the recurrence runs up to degree N, that systematic error dominates.
// Each point is therefore carried as a double-double x_hi + x_lo (or
// (x - x0)_hi + (x - x0)_lo), built from the exact rational angle, and every
// step forms A_n x u as A_n (x_hi u + x_lo u): rounding the linear factor
// A_n x + B_n to FP64 first would act like a rounded point again (it costs
// about a factor 10 in the inverse when the recurrence covers the whole
// matrix).  What remains is the per-step rounding of the recurrence itself.
#include "cjt_internal.h"

namespace cjt {

// ------------------------------------------------------------------ points

namespace {

struct ddv {
    double hi, lo;
};

__device__ __forceinline__ ddv fast_two_sum(double a, double b)
{
#pragma clang fp contract(off)
    const double s = a + b;
    return {s, b - (s - a)};
}

__device__ __forceinline__ ddv dd_add(ddv a, ddv b)
{
#pragma clang fp contract(off)
    const double s = a.hi + b.hi;
    const double bb = s - a.hi;
    const double e = (a.hi - (s - bb)) + (b.hi - bb);
    return fast_two_sum(s, e + a.lo + b.lo);
}

__device__ __forceinline__ ddv dd_mul(ddv a, ddv b)
{
#pragma clang fp contract(off)
    const double p = a.hi * b.hi;
    const double e = fma(a.hi, b.hi, -p);
    return fast_two_sum(p, fma(a.hi, b.lo, fma(a.lo, b.hi, e)));
}

// a / m for an integer m < 2^53
__device__ __forceinline__ ddv dd_div(ddv a, double m)
{
#pragma clang fp contract(off)
    const double q = a.hi / m;
    const double r = fma(-q, m, a.hi) + a.lo;
    return fast_two_sum(q, r / m);
}

// sin(pi num / den) for integers |num| <= den / 4, den < 2^53, in double-double:
// the ratio is formed exactly, multiplied by pi (double-double), and the
// Taylor series is summed by Horner's rule, 14 terms (the first omitted term
// is below 1e-33 of the result for |angle| <= pi/4).
__device__ ddv sinpi_ratio(double num, double den)
{
#pragma clang fp contract(off)
    const double fh = num / den;
    const ddv f = fast_two_sum(fh, fma(-fh, den, num) / den);
    const ddv pi = {3.141592653589793116e+00, 1.2246467991473532072e-16};
    const ddv a = dd_mul(pi, f);
    const ddv a2 = dd_mul(a, a);
    ddv s = {1.0, 0.0};
    for (int k = 13; k >= 1; --k) {
        const ddv t = dd_div(dd_mul(a2, s), (double)(2 * k) * (double)(2 * k + 1));
        s = dd_add(ddv{1.0, 0.0}, ddv{-t.hi, -t.lo});
    }
    return dd_mul(a, s);
}

// Point i of the grid theta_i = pi i / G: x_i (mode 0, pi/4 <= theta <= 3pi/4),
// x_i - 1 = -2 sin^2(theta/2) (mode +1) or x_i + 1 = 2 sin^2((pi - theta)/2)
// (mode -1), as hi + lo.
__device__ void grid_point(int64_t i, int64_t G, int mode, double& hi, double& lo)
{
    ddv v;
    if (mode == 0) {
        v = sinpi_ratio((double)(G - 2 * i), (double)(2 * G));
    } else {
        const ddv sh = sinpi_ratio((double)(mode > 0 ? i : G - i), (double)(2 * G));
        v = dd_mul(sh, sh);
        const double sc = mode > 0 ? -2.0 : 2.0;
        v = {v.hi * sc, v.lo * sc};
    }
    hi = v.hi;
    lo = v.lo;
}

}  // namespace

constexpr int kPPT = 4;     // points per thread, inverse
constexpr int kChunk = 16;  // degrees per LDS reduction round (divides kBlk)

// ------------------------------------------------------------------ forward

// Each lane carries kPPTF points of the task (up to 64*kPPTF points, one
// recurrence per point).  The per-degree coefficients (a d4 record and c_n)
// are staged through LDS in blocks of kBlk degrees with coalesced vector
// loads; the loads of the next block are issued before the current block is
// consumed, so the serial chain never waits on memory latency.
constexpr int kPPTF = 4;
constexpr int kBlk = 128;

struct Stage {
    d4 co[kBlk];
    double c[kBlk];
};

// Global -> registers for degrees [n0, n0 + kBlk) (clipped to [lo, hi)): lane l
// takes degrees n0 + l and n0 + l + 64.
struct StageRegs {
    d4 co[2];
    double c[2];
};

__device__ __forceinline__ void stage_load(StageRegs& r, const d4* __restrict__ co, const double* __restrict__ c,
                                           int n0, int lo, int hi, int lane)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int n = n0 + lane + 64 * h;
        if (n >= lo && n < hi) {
            r.co[h] = co[n];
            r.c[h] = c ? c[n] : 0.0;
        } else {
            r.co[h] = d4{0.0, 0.0, 0.0, 0.0};
            r.c[h] = 0.0;
        }
    }
}

__device__ __forceinline__ void stage_store(Stage& st, const StageRegs& r, int lane)
{
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        st.co[lane + 64 * h] = r.co[h];
        st.c[lane + 64 * h] = r.c[h];
    }
}

__global__ void __launch_bounds__(64) k_rec_fwd(const ExecDesc* __restrict__ descs)
{
    __shared__ Stage stg[2];
    const ExecDesc& d = descs[blockIdx.x];
    const int task = blockIdx.y;
    if (task >= d.ntasks) return;
    cptr<RecTask> tp = as_const(d.tasks) + task;
    const int p0 = uniform(tp->p0), np = uniform(tp->np), mode = uniform(tp->mode), cut = uniform(tp->cut);
    const int lane = threadIdx.x;
    const int64_t N = d.N;
    const double* __restrict__ c = d.in;
    const d4* __restrict__ co = mode == 0 ? d.rec0 : (mode > 0 ? d.recp : d.recm);
    // plain: (A_n, B_n, C_{n+1});  modified: (A_n, C_{n+1} r_{n+1}, 1/r_n)
    double xh[kPPTF], xl[kPPTF], s1[kPPTF], s2[kPPTF];
    for (int q = 0; q < kPPTF; ++q) {
        const int idx = lane + 64 * q;
        const int64_t i = p0 + (idx < np ? idx : 0);
        grid_point(i, N, mode, xh[q], xl[q]);
        s1[q] = 0.0;  // plain: u_{n+1};  modified: u_{n+1}
        s2[q] = 0.0;  // plain: u_{n+2};  modified: D_{n+1}
    }
    // blocks cover [b0, b0 + kBlk) with b0 descending from the top
    const int nblk = (cut + kBlk - 1) / kBlk;
    StageRegs rg;
    int buf = 0;
    if (nblk > 0) {
        stage_load(rg, co, c, (nblk - 1) * kBlk, 0, cut, lane);
        stage_store(stg[0], rg, lane);
    }
    __syncthreads();
    for (int b = nblk - 1; b >= 0; --b) {
        const int b0 = b * kBlk;
        if (b > 0) stage_load(rg, co, c, b0 - kBlk, 0, cut, lane);
        const Stage& S = stg[buf];
        const int top = min(kBlk, cut - b0) - 1;
        if (mode == 0) {
#pragma unroll 8
            for (int t = top; t >= 0; --t) {
                const d4 q4 = S.co[t];
                const double cn = S.c[t];
#pragma unroll
                for (int q = 0; q < kPPTF; ++q) {
                    const double w = fma(xh[q], s1[q], xl[q] * s1[q]);
                    const double u0 = fma(q4.x, w, fma(q4.y, s1[q], fma(-q4.z, s2[q], cn)));
                    s2[q] = s1[q];
                    s1[q] = u0;
                }
            }
        } else {
#pragma unroll 8
            for (int t = top; t >= 0; --t) {
                const d4 q4 = S.co[t];
                const double cn = S.c[t];
                const bool last = (b0 + t) == 0;
#pragma unroll
                for (int q = 0; q < kPPTF; ++q) {
                    const double w = fma(xh[q], s1[q], xl[q] * s1[q]);
                    const double Dn = fma(q4.x, w, fma(q4.y, s2[q], cn));
                    if (!last) s1[q] = fma(s1[q], q4.z, Dn);
                    s2[q] = Dn;
                }
            }
        }
        if (b > 0) stage_store(stg[buf ^ 1], rg, lane);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int q = 0; q < kPPTF; ++q) {
        const int idx = lane + 64 * q;
        if (idx < np) d.p[p0 + idx] = mode == 0 ? s1[q] : s2[q];
    }
}

cjt_status launch_rec_fwd(const EngineArgs& a)
{
    if (a.count <= 0 || a.max_tasks <= 0) return CJT_OK;
    dim3 grid(a.count, a.max_tasks);
    hipLaunchKernelGGL(k_rec_fwd, grid, dim3(64), 0, a.stream, a.d_desc);
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

// ------------------------------------------------------------------ inverse

__global__ void __launch_bounds__(64) k_rec_inv(const ExecDesc* __restrict__ descs)
{
    __shared__ double red[kChunk][64 + 1];
    __shared__ Stage stg[2];
    const ExecDesc& d = descs[blockIdx.x];
    const int task = blockIdx.y;
    if (task >= d.ntasks) return;
    cptr<RecTask> tp = as_const(d.tasks) + task;
    const int p0 = uniform(tp->p0), np = uniform(tp->np), mode = uniform(tp->mode), cut = uniform(tp->cut);
    const int64_t off = tp->off;
    const int lane = threadIdx.x;
    const int64_t G = d.G;
    double* __restrict__ part = d.part + off;

    double pv[kPPT], ev[kPPT], xh[kPPT], xl[kPPT];
    for (int q = 0; q < kPPT; ++q) {
        const int idx = lane + 64 * q;
        const bool act = idx < np;
        const int64_t j = p0 + (act ? idx : 0);
        const double g = act ? d.p[j] : 0.0;
        pv[q] = g;      // pi_0 = g_j (scaled recurrence)
        ev[q] = 0.0;    // e_0 = 0 (modified) / P_{-1} = 0 (three-term)
        grid_point(j, G, mode, xh[q], xl[q]);
    }
    // three-term: (A_n, B_n, C_n);  modified: (A_n, C_n / r_{n-1}, r_n)
    const d4* __restrict__ co = mode == 0 ? d.rec0 : (mode > 0 ? d.recp : d.recm);
    const int dd = lane >> 2, qq = lane & 3;  // reduction: degree dd of the chunk, quarter qq of the 64 lanes
    const int nblk = (cut + kBlk - 1) / kBlk;
    StageRegs rg;
    int buf = 0;
    if (nblk > 0) {
        stage_load(rg, co, nullptr, 0, 0, cut, lane);
        stage_store(stg[0], rg, lane);
    }
    __syncthreads();
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * kBlk;
        if (b + 1 < nblk) stage_load(rg, co, nullptr, b0 + kBlk, 0, cut, lane);
        const Stage& S = stg[buf];
        const int bend = min(kBlk, cut - b0);
        for (int c0 = 0; c0 < bend; c0 += kChunk) {
            const int nend = min(kChunk, bend - c0);
#pragma unroll 8
            for (int t = 0; t < nend; ++t) {
                double v = 0.0;
#pragma unroll
                for (int q = 0; q < kPPT; ++q) v += pv[q];
                red[t][lane] = v;
                const d4 cf = S.co[c0 + t];
                if (mode == 0) {
#pragma unroll
                    for (int q = 0; q < kPPT; ++q) {
                        const double w = fma(xh[q], pv[q], xl[q] * pv[q]);
                        const double p1 = fma(cf.x, w, fma(cf.y, pv[q], -cf.z * ev[q]));
                        ev[q] = pv[q];
                        pv[q] = p1;
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < kPPT; ++q) {
                        const double w = fma(xh[q], pv[q], xl[q] * pv[q]);
                        const double e1 = fma(cf.x, w, cf.y * ev[q]);
                        pv[q] = fma(pv[q], cf.z, e1);
                        ev[q] = e1;
                    }
                }
            }
            __syncthreads();
            if (dd < nend) {
                double sum = 0.0;
#pragma unroll
                for (int l = 0; l < 16; ++l) sum += red[dd][qq * 16 + l];
                sum += __shfl_xor(sum, 1);
                sum += __shfl_xor(sum, 2);
                if (qq == 0) part[b0 + c0 + dd] = sum;
            }
            __syncthreads();
        }
        if (b + 1 < nblk) stage_store(stg[buf ^ 1], rg, lane);
        __syncthreads();
        buf ^= 1;
    }
}

cjt_status launch_rec_inv(const EngineArgs& a)
{
    if (a.count <= 0 || a.max_tasks <= 0) return CJT_OK;
    dim3 grid(a.count, a.max_tasks);
    hipLaunchKernelGGL(k_rec_inv, grid, dim3(64), 0, a.stream, a.d_desc);
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

// out[n] = s_n (out[n] + sum over tasks t with cut_t > n of part_t[n]); tasks
// are sorted by decreasing cut, so they form a prefix.
__global__ void __launch_bounds__(256) k_rec_inv_reduce(const ExecDesc* __restrict__ descs)
{
    const ExecDesc& d = descs[blockIdx.y];
    const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (n > d.N) return;
    double acc = 0.0;
    cptr<RecTask> tasks = as_const(d.tasks);
    for (int t = 0; t < d.ntasks; ++t) {
        const int cut = tasks[t].cut;
        if (cut <= n) break;
        acc += d.part[tasks[t].off + n];
    }
    d.out[n] = d.s[n] * (d.out[n] + acc);
}

cjt_status launch_rec_inv_reduce(const EngineArgs& a, int64_t maxN)
{
    if (a.count <= 0) return CJT_OK;
    dim3 grid((unsigned)((maxN + 1 + 255) / 256), a.count);
    hipLaunchKernelGGL(k_rec_inv_reduce, grid, dim3(256), 0, a.stream, a.d_desc);
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

}  // namespace cjt
