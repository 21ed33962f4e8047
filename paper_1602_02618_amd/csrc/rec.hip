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
#include <stdlib.h>

#include <algorithm>
#include <cmath>

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

constexpr int kPPT = 4;     // points per lane (tasks are at most 64 * kPPT points)
constexpr int kChunk = 16;  // degrees per LDS reduction round (divides kBlk)
constexpr int kBlk = 128;   // degrees per LDS coefficient block
constexpr int kRec = 6 * 64 * kPPT;  // doubles per segment record (6 per point)

// ------------------------------------------------------------------ segments
//
// A task whose degree range [0, cut) is long would be one serial chain of cut
// steps.  With a segment length S (chosen per call from the total work), a
// task with cut > 2S is split into nseg = ceil(cut / S) segments of equal
// length (rounded up to kBlk).  Every recurrence here is linear in its
// two-term state, so a segment maps the state entering it to the state
// leaving it by an affine map (forward: Clenshaw run downward, with the
// coefficients c_n) or a linear one (inverse: the recurrence run upward).
// Segments compute their maps in parallel (two extra homogeneous chains),
// and a short serial pass per point chains them.

__host__ __device__ __forceinline__ int seg_count(int cut, int S) { return cut > S ? (cut + S - 1) / S : 1; }

__host__ __device__ __forceinline__ int seg_len(int cut, int nseg)
{
    const int l = (cut + nseg - 1) / nseg;
    return (l + kBlk - 1) / kBlk * kBlk;
}

// ------------------------------------------------------------------ coefficient staging
//
// The per-degree coefficients (a d4 record and c_n) are staged through LDS in
// blocks of kBlk degrees with coalesced vector loads; the loads of the next
// block are issued before the current block is consumed, so the serial chain
// never waits on memory latency.

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
            r.co[h] = ldg(co + n);
            r.c[h] = c ? ldg(c + n) : 0.0;
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

struct TaskView {
    int p0, np, mode, cut;
    int64_t off;
};

__device__ __forceinline__ TaskView task_of(const ExecDesc& d, int t)
{
    cptr<RecTask> tp = as_const(d.tasks) + t;
    return TaskView{uniform(tp->p0), uniform(tp->np), uniform(tp->mode), uniform(tp->cut), tp->off};
}

// ------------------------------------------------------------------ forward

// Item (desc, task, segment, record slot).  kSplit = false: the whole range
// [0, cut) of the task, result written to p.  kSplit = true: one segment;
// chain 0 runs from a zero state with c_n (the affine part), chains 1 and 2
// from the unit states without c_n (the linear part); the three final states
// go to the segment's record.
template <bool kSplit>
__global__ void __launch_bounds__(64) k_rec_fwd(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    __shared__ Stage sbuf[2];
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const TaskView tk = task_of(d, it.a);
    const int lane = threadIdx.x;
    int lo = 0, hi = tk.cut;
    if (kSplit) {
        const int S = d.rec_seg;
        const int sl = seg_len(tk.cut, seg_count(tk.cut, S));
        lo = it.b * sl;
        hi = min(tk.cut, lo + sl);
    }
    const int mode = tk.mode;
    const d4* __restrict__ co = mode == 0 ? d.rec0 : (mode > 0 ? d.recp : d.recm);
    constexpr int NC = kSplit ? 3 : 1;
    // plain: (A_n, B_n, C_{n+1});  modified: (A_n, C_{n+1} r_{n+1}, 1/r_n)
    double xh[kPPT], xl[kPPT], s1[NC][kPPT], s2[NC][kPPT];
    for (int q = 0; q < kPPT; ++q) {
        const int idx = lane + 64 * q;
        const int64_t i = tk.p0 + (idx < tk.np ? idx : 0);
        grid_point(i, d.N, mode, xh[q], xl[q]);
#pragma unroll
        for (int ch = 0; ch < NC; ++ch) {
            s1[ch][q] = ch == 1 ? 1.0 : 0.0;  // plain: u_{n+1};  modified: u_{n+1}
            s2[ch][q] = ch == 2 ? 1.0 : 0.0;  // plain: u_{n+2};  modified: D_{n+1}
        }
    }
    // blocks cover [lo + b kBlk, ...) with b descending from the top
    const int nb = (hi - lo + kBlk - 1) / kBlk;
    StageRegs rg;
    int buf = 0;
    if (nb > 0) {
        stage_load(rg, co, d.in, lo + (nb - 1) * kBlk, lo, hi, lane);
        stage_store(sbuf[0], rg, lane);
    }
    __syncthreads();
    for (int b = nb - 1; b >= 0; --b) {
        const int b0 = lo + b * kBlk;
        if (b > 0) stage_load(rg, co, d.in, b0 - kBlk, lo, hi, lane);
        const Stage& St = sbuf[buf];
        const int top = min(kBlk, hi - b0) - 1;
        if (mode == 0) {
#pragma unroll 4
            for (int t = top; t >= 0; --t) {
                const d4 q4 = St.co[t];
                const double cn = St.c[t];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                    for (int q = 0; q < kPPT; ++q) {
                        const double w = fma(xh[q], s1[ch][q], xl[q] * s1[ch][q]);
                        const double u0 = fma(q4.x, w, fma(q4.y, s1[ch][q], fma(-q4.z, s2[ch][q], ch == 0 ? cn : 0.0)));
                        s2[ch][q] = s1[ch][q];
                        s1[ch][q] = u0;
                    }
            }
        } else {
            // degree 0 ends the modified recurrence without the u update; it
            // is taken after the loop so the loop body carries no such test
            const int stop = b0 == 0 ? 1 : 0;
#pragma unroll 4
            for (int t = top; t >= stop; --t) {
                const d4 q4 = St.co[t];
                const double cn = St.c[t];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                    for (int q = 0; q < kPPT; ++q) {
                        const double w = fma(xh[q], s1[ch][q], xl[q] * s1[ch][q]);
                        const double Dn = fma(q4.x, w, fma(q4.y, s2[ch][q], ch == 0 ? cn : 0.0));
                        s1[ch][q] = fma(s1[ch][q], q4.z, Dn);
                        s2[ch][q] = Dn;
                    }
            }
            if (b0 == 0) {
                const d4 q4 = St.co[0];
                const double cn = St.c[0];
#pragma unroll
                for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                    for (int q = 0; q < kPPT; ++q) {
                        const double w = fma(xh[q], s1[ch][q], xl[q] * s1[ch][q]);
                        s2[ch][q] = fma(q4.x, w, fma(q4.y, s2[ch][q], ch == 0 ? cn : 0.0));
                    }
            }
        }
        if (b > 0) stage_store(sbuf[buf ^ 1], rg, lane);
        __syncthreads();
        buf ^= 1;
    }
    if (!kSplit) {
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
            const int idx = lane + 64 * q;
            if (idx < tk.np) stg(d.p + tk.p0 + idx, mode == 0 ? s1[0][q] : s2[0][q]);
        }
    } else {
        double* rec = d.seg + (int64_t)it.c * kRec;
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
            const int idx = lane + 64 * q;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) {
                stg(rec + (2 * ch) * 64 * kPPT + idx, s1[ch][q]);
                stg(rec + (2 * ch + 1) * 64 * kPPT + idx, s2[ch][q]);
            }
        }
    }
}

// Item (desc, task, nseg, first slot): state (u, s2) entering the top segment
// is zero; each segment, from the top, maps it to
//     state' = affine + u * unit1 + s2 * unit2,
// and the bottom segment's result is u_0 (three-term) or D_0 (modified).
__global__ void __launch_bounds__(64) k_rec_fwd_combine(const ExecDesc* __restrict__ descs,
                                                        const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const TaskView tk = task_of(d, it.a);
    const int nseg = it.b;
    constexpr int R = 64 * kPPT;
    for (int q = 0; q < kPPT; ++q) {
        const int idx = threadIdx.x + 64 * q;
        double x = 0.0, y = 0.0;
#pragma unroll 4
        for (int s = nseg - 1; s >= 0; --s) {
            const double* rec = d.seg + (int64_t)(it.c + s) * kRec + idx;
            const double nx = ldg(rec) + fma(ldg(rec + 2 * R), x, ldg(rec + 4 * R) * y);
            const double ny = ldg(rec + R) + fma(ldg(rec + 3 * R), x, ldg(rec + 5 * R) * y);
            x = nx;
            y = ny;
        }
        if (idx < tk.np) stg(d.p + tk.p0 + idx, tk.mode == 0 ? x : y);
    }
}

// ------------------------------------------------------------------ inverse

// Item (desc, task, segment, record slot), degrees [lo, hi) of the task.
// kMaps: the two unit states are run through the segment and the final
// states stored (records 0..3).  Otherwise the state entering the segment is
// (g_j, 0) for an unsplit task or records 4, 5 of the slot, and each degree's
// values are summed over the task's points into part[off + n].
template <bool kMaps>
__global__ void __launch_bounds__(64) k_rec_inv(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    __shared__ double red[kChunk][64 + 1];
    __shared__ Stage sbuf[2];
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const TaskView tk = task_of(d, it.a);
    const int lane = threadIdx.x;
    const int64_t G = d.G;
    const bool split = it.c >= 0;
    int lo = 0, hi = tk.cut;
    if (split) {
        const int S = d.rec_seg;
        const int sl = seg_len(tk.cut, seg_count(tk.cut, S));
        lo = it.b * sl;
        hi = min(tk.cut, lo + sl);
    }
    const int mode = tk.mode;
    double* __restrict__ part = d.part + tk.off;
    constexpr int NC = kMaps ? 2 : 1;
    constexpr int R = 64 * kPPT;
    double* rec = split ? d.seg + (int64_t)it.c * kRec : nullptr;

    double pv[NC][kPPT], ev[NC][kPPT], xh[kPPT], xl[kPPT];
    for (int q = 0; q < kPPT; ++q) {
        const int idx = lane + 64 * q;
        const bool act = idx < tk.np;
        const int64_t j = tk.p0 + (act ? idx : 0);
        if (kMaps) {
            pv[0][q] = 1.0;
            ev[0][q] = 0.0;
            pv[NC - 1][q] = 0.0;
            ev[NC - 1][q] = 1.0;
        } else if (split) {
            pv[0][q] = ldg(rec + 4 * R + idx);
            ev[0][q] = ldg(rec + 5 * R + idx);
        } else {
            pv[0][q] = act ? ldg(d.p + j) : 0.0;  // pi_0 = g_j (scaled recurrence)
            ev[0][q] = 0.0;                 // e_0 = 0 (modified) / P_{-1} = 0 (three-term)
        }
        grid_point(j, G, mode, xh[q], xl[q]);
    }
    // three-term: (A_n, B_n, C_n);  modified: (A_n, C_n / r_{n-1}, r_n)
    const d4* __restrict__ co = mode == 0 ? d.rec0 : (mode > 0 ? d.recp : d.recm);
    const int dd = lane >> 2, qq = lane & 3;  // reduction: degree dd of the chunk, quarter qq of the 64 lanes
    const int nb = (hi - lo + kBlk - 1) / kBlk;
    StageRegs rg;
    int buf = 0;
    if (nb > 0) {
        stage_load(rg, co, nullptr, lo, lo, hi, lane);
        stage_store(sbuf[0], rg, lane);
    }
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
        const int b0 = lo + b * kBlk;
        if (b + 1 < nb) stage_load(rg, co, nullptr, b0 + kBlk, lo, hi, lane);
        const Stage& St = sbuf[buf];
        const int bend = min(kBlk, hi - b0);
        for (int c0 = 0; c0 < bend; c0 += kChunk) {
            const int nend = min(kChunk, bend - c0);
            // this lane's points summed at each degree (the first point starts
            // the sum), for the reduction below
            auto put = [&](int t) {
                if (!kMaps) {
                    double v = pv[0][0];
#pragma unroll
                    for (int q = 1; q < kPPT; ++q) v += pv[0][q];
                    red[t][lane] = v;
                }
            };
            // one loop per form (the form is fixed for the task), so the
            // unrolled body carries no branch
            if (mode == 0) {
#pragma unroll 4
                for (int t = 0; t < nend; ++t) {
                    put(t);
                    const d4 cf = St.co[c0 + t];
#pragma unroll
                    for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                        for (int q = 0; q < kPPT; ++q) {
                            const double w = fma(xh[q], pv[ch][q], xl[q] * pv[ch][q]);
                            const double p1 = fma(cf.x, w, fma(cf.y, pv[ch][q], -cf.z * ev[ch][q]));
                            ev[ch][q] = pv[ch][q];
                            pv[ch][q] = p1;
                        }
                }
            } else {
#pragma unroll 4
                for (int t = 0; t < nend; ++t) {
                    put(t);
                    const d4 cf = St.co[c0 + t];
#pragma unroll
                    for (int ch = 0; ch < NC; ++ch)
#pragma unroll
                        for (int q = 0; q < kPPT; ++q) {
                            const double w = fma(xh[q], pv[ch][q], xl[q] * pv[ch][q]);
                            const double e1 = fma(cf.x, w, cf.y * ev[ch][q]);
                            pv[ch][q] = fma(pv[ch][q], cf.z, e1);
                            ev[ch][q] = e1;
                        }
                }
            }
            if (!kMaps) {
                __syncthreads();
                if (dd < nend) {
                    double sum = red[dd][qq * 16];
#pragma unroll
                    for (int l = 1; l < 16; ++l) sum += red[dd][qq * 16 + l];
                    sum += __shfl_xor(sum, 1);
                    sum += __shfl_xor(sum, 2);
                    if (qq == 0) stg(part + b0 + c0 + dd, sum);
                }
                __syncthreads();
            }
        }
        if (b + 1 < nb) stage_store(sbuf[buf ^ 1], rg, lane);
        __syncthreads();
        buf ^= 1;
    }
    if (kMaps) {
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
            const int idx = lane + 64 * q;
#pragma unroll
            for (int ch = 0; ch < NC; ++ch) {
                stg(rec + (2 * ch) * R + idx, pv[ch][q]);
                stg(rec + (2 * ch + 1) * R + idx, ev[ch][q]);
            }
        }
    }
}

// Item (desc, task, nseg, first slot): starting state of every segment,
// (g_j, 0) at degree 0, then each segment's linear map (records 0..3).
__global__ void __launch_bounds__(64) k_rec_inv_init(const ExecDesc* __restrict__ descs,
                                                     const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const TaskView tk = task_of(d, it.a);
    const int nseg = it.b;
    constexpr int R = 64 * kPPT;
    // The records hold maps (0..3) and start states (4, 5) in disjoint
    // slots, but the compiler cannot see that: a load placed after a store
    // waits for it.  So each segment's maps are loaded one step ahead, before
    // the current states are stored, and the lane's points (independent
    // chains) step together.
    double x[kPPT], y[kPPT], a[kPPT], b[kPPT], c[kPPT], e[kPPT];
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
        const int idx = threadIdx.x + 64 * q;
        x[q] = idx < tk.np ? ldg(d.p + tk.p0 + idx) : 0.0;
        y[q] = 0.0;
        const double* r = d.seg + (int64_t)it.c * kRec + idx;
        a[q] = ldg(r);
        b[q] = ldg(r + R);
        c[q] = ldg(r + 2 * R);
        e[q] = ldg(r + 3 * R);
    }
    for (int s = 0; s < nseg; ++s) {
        double* rec = d.seg + (int64_t)(it.c + s) * kRec + threadIdx.x;
        const bool more = s + 1 < nseg;
        double na[kPPT], nb[kPPT], nc[kPPT], ne[kPPT];
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
            // the next segment's maps (record s + 1 exists while s + 1 < nseg;
            // the last step re-reads this record's maps, unused)
            const double* r = rec + (more ? kRec : 0) + 64 * q;
            na[q] = ldg(r);
            nb[q] = ldg(r + R);
            nc[q] = ldg(r + 2 * R);
            ne[q] = ldg(r + 3 * R);
        }
#pragma unroll
        for (int q = 0; q < kPPT; ++q) {
            stg(rec + 64 * q + 4 * R, x[q]);
            stg(rec + 64 * q + 5 * R, y[q]);
            const double nx = fma(a[q], x[q], c[q] * y[q]);
            const double ny = fma(b[q], x[q], e[q] * y[q]);
            x[q] = nx;
            y[q] = ny;
            a[q] = na[q];
            b[q] = nb[q];
            c[q] = nc[q];
            e[q] = ne[q];
        }
    }
}

// out[n] = s_n (Hahn part + sum over tasks t with cut_t > n of part_t[n]).
// Item (desc, tile of 256/GR degrees); GR groups of lanes split the tasks
// (t = group mod GR) and are added in a fixed order (GR = 8 for instances
// with many tasks, 1 otherwise).  Tasks are sorted by decreasing cut, so the
// contributing ones form a prefix.
template <int GR>
__global__ void __launch_bounds__(256) k_rec_inv_reduce(const ExecDesc* __restrict__ descs,
                                                        const Item* __restrict__ items)
{
    constexpr int DN = 256 / GR;  // degrees per workgroup
    __shared__ double red[GR][DN + 1];
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const int dn = threadIdx.x % DN, grp = threadIdx.x / DN;
    const int64_t n = (int64_t)it.b * DN + dn;
    int lo = 0, hi = d.ntasks;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ldg(&d.tasks[mid].cut) > n) lo = mid + 1;
        else hi = mid;
    }
    const int T = lo;
    double acc = 0.0;
#pragma unroll 4
    for (int t = grp; t < T; t += GR) acc += ldg(d.part + ldg(&d.tasks[t].off) + n);
    red[grp][dn] = acc;
    __syncthreads();
    if (grp == 0 && n <= d.N) {
        double tot = 0.0;
#pragma unroll
        for (int g = 0; g < GR; ++g) tot += red[g][dn];
        const double base = d.nblk > 0 ? ldg(d.out + n) : 0.0;
        stg(d.out + n, ldg(d.s + n) * (base + tot));
    }
}

// ------------------------------------------------------------------ host side

int32_t rec_segment_length(const Program& pr, const std::vector<const RecTask*>& tasks, const std::vector<int>& which)
{
    if (const char* e = getenv("CJT_REC_SEGMENT")) {
        const int v = atoi(e);
        if (v > 0) return std::max(kBlk, (v + kBlk - 1) / kBlk * kBlk);
    }
    // total chain steps W: with one wave per SIMD busy on FP64 issue, the
    // recurrence phase takes about W / 1024 steps of time; a chain longer than
    // that would be the critical path, so chains are cut to that share, but
    // never below one coefficient block (single transforms of N = 1024 measured
    // 155 us at a 256-step floor and 114 us at 128)
    double W = 0.0;
    for (int i : which)
        for (int t = 0; t < pr.descs[i].ntasks; ++t) W += (double)tasks[i][t].cut;
    const double S = std::max((double)kBlk, std::ceil(W / 1024.0));
    const int Si = (int)std::min(S, 1.0e9);
    return (Si + kBlk - 1) / kBlk * kBlk;
}

int64_t rec_seg_doubles(const ExecDesc& d, const RecTask* tasks)
{
    int64_t slots = 0;
    for (int t = 0; t < d.ntasks; ++t) {
        const int ns = seg_count(tasks[t].cut, d.rec_seg);
        if (ns > 1) slots += ns;
    }
    return slots * kRec;
}

namespace {

Launch rec_launch(Kind k, int stream, int nth, const char* name, double flops, double bytes)
{
    Launch L;
    L.kind = k;
    L.stream = stream;
    L.nth = nth;
    L.name = name;
    L.flops = flops;
    L.bytes = bytes;
    return L;
}

// Longest chains first over the whole call, so that no long chain of a late
// instance starts after the short ones have drained (ties keep their order).
void by_length(std::vector<Item>& items, const Program& pr, const std::vector<const RecTask*>& tasks)
{
    auto len = [&](const Item& it) {
        const int cut = tasks[it.desc][it.a].cut;
        const int ns = seg_count(cut, pr.descs[it.desc].rec_seg);
        return ns == 1 ? cut : seg_len(cut, ns);
    };
    std::stable_sort(items.begin(), items.end(), [&](const Item& x, const Item& y) { return len(x) > len(y); });
}

void push(Program& pr, Launch L, const std::vector<Item>& items)
{
    if (items.empty()) return;
    L.item_off = (int64_t)pr.items.size();
    L.nitems = (int64_t)items.size();
    pr.items.insert(pr.items.end(), items.begin(), items.end());
    pr.launches.push_back(L);
}

}  // namespace

void add_rec_fwd(Program& pr, const std::vector<const RecTask*>& tasks, int stream, double flops, double bytes)
{
    std::vector<Item> whole, segs, comb;
    for (size_t i = 0; i < pr.descs.size(); ++i) {
        int slot = 0;
        for (int t = 0; t < pr.descs[i].ntasks; ++t) {
            const int ns = seg_count(tasks[i][t].cut, pr.descs[i].rec_seg);
            if (tasks[i][t].cut <= 0) continue;
            if (ns == 1) {
                whole.push_back(Item{(int32_t)i, t, 0, -1});
            } else {
                for (int s = 0; s < ns; ++s) segs.push_back(Item{(int32_t)i, t, s, slot + s});
                comb.push_back(Item{(int32_t)i, t, ns, slot});
                slot += ns;
            }
        }
    }
    by_length(segs, pr, tasks);
    by_length(whole, pr, tasks);
    push(pr, rec_launch(Kind::RecFwdSeg, stream, 64, "rec_forward", flops * 0.5, bytes * 0.5), segs);
    push(pr, rec_launch(Kind::RecFwd, stream, 64, "rec_forward", segs.empty() ? flops : flops * 0.5,
                        segs.empty() ? bytes : bytes * 0.5),
         whole);
    push(pr, rec_launch(Kind::RecFwdCombine, stream, 64, "rec_forward_combine", 0.0, 0.0), comb);
}

void add_rec_inv(Program& pr, const std::vector<const RecTask*>& tasks, int stream, double flops, double bytes)
{
    std::vector<Item> maps, init, all;
    for (size_t i = 0; i < pr.descs.size(); ++i) {
        int slot = 0;
        for (int t = 0; t < pr.descs[i].ntasks; ++t) {
            if (tasks[i][t].cut <= 0) continue;
            const int ns = seg_count(tasks[i][t].cut, pr.descs[i].rec_seg);
            if (ns == 1) {
                all.push_back(Item{(int32_t)i, t, 0, -1});
            } else {
                for (int s = 0; s < ns; ++s) {
                    if (s + 1 < ns) maps.push_back(Item{(int32_t)i, t, s, slot + s});
                    all.push_back(Item{(int32_t)i, t, s, slot + s});
                }
                init.push_back(Item{(int32_t)i, t, ns, slot});
                slot += ns;
            }
        }
    }
    by_length(maps, pr, tasks);
    by_length(all, pr, tasks);
    push(pr, rec_launch(Kind::RecInvMaps, stream, 64, "rec_inverse_maps", 0.0, 0.0), maps);
    push(pr, rec_launch(Kind::RecInvInit, stream, 64, "rec_inverse_init", 0.0, 0.0), init);
    push(pr, rec_launch(Kind::RecInv, stream, 64, "rec_inverse", flops, bytes), all);
}

void add_rec_inv_reduce(Program& pr, int stream, double bytes)
{
    // many tasks per degree (large N): eight groups share them; otherwise one
    std::vector<Item> wide, narrow;
    for (size_t i = 0; i < pr.descs.size(); ++i) {
        const bool many = pr.descs[i].ntasks >= 1024;
        const int dn = many ? 32 : 256;
        for (int64_t t = 0; t < (pr.descs[i].N + 1 + dn - 1) / dn; ++t)
            (many ? wide : narrow).push_back(Item{(int32_t)i, 0, (int32_t)t, 0});
    }
    const double tot = (double)(wide.size() * 32 + narrow.size() * 256);
    Launch L = rec_launch(Kind::RecInvReduce, stream, 256, "rec_inverse_reduce", 0.0, 0.0);
    L.acc_off = 8;  // groups
    L.bytes = tot > 0 ? bytes * (double)(wide.size() * 32) / tot : 0.0;
    push(pr, L, wide);
    L.acc_off = 1;
    L.bytes = tot > 0 ? bytes * (double)(narrow.size() * 256) / tot : 0.0;
    push(pr, L, narrow);
}

cjt_status launch_rec(const Launch& L, const ExecDesc* dd, const Item* it, hipStream_t s)
{
    if (L.nitems <= 0) return CJT_OK;
    ProfScope ps(L.name, L.flops, L.bytes, s);
    const dim3 grid((unsigned)L.nitems), block(L.nth);
    switch (L.kind) {
    case Kind::RecFwd: hipLaunchKernelGGL(k_rec_fwd<false>, grid, block, 0, s, dd, it); break;
    case Kind::RecFwdSeg: hipLaunchKernelGGL(k_rec_fwd<true>, grid, block, 0, s, dd, it); break;
    case Kind::RecFwdCombine: hipLaunchKernelGGL(k_rec_fwd_combine, grid, block, 0, s, dd, it); break;
    case Kind::RecInvMaps: hipLaunchKernelGGL(k_rec_inv<true>, grid, block, 0, s, dd, it); break;
    case Kind::RecInvInit: hipLaunchKernelGGL(k_rec_inv_init, grid, block, 0, s, dd, it); break;
    case Kind::RecInv: hipLaunchKernelGGL(k_rec_inv<false>, grid, block, 0, s, dd, it); break;
    case Kind::RecInvReduce:
        if (L.acc_off == 8) hipLaunchKernelGGL(k_rec_inv_reduce<8>, grid, block, 0, s, dd, it);
        else hipLaunchKernelGGL(k_rec_inv_reduce<1>, grid, block, 0, s, dd, it);
        break;
    default: return fail(CJT_EINVAL, "not a recurrence launch");
    }
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

}  // namespace cjt
