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
#include "cjt_internal.h"

namespace cjt {

constexpr int kPPT = 4;     // points per thread, inverse
constexpr int kChunk = 16;  // degrees per LDS reduction round

// ------------------------------------------------------------------ forward

// Each lane carries kPPTF points of the task (up to 64*kPPTF points, one
// recurrence per point); coefficients are loaded once per degree for all of
// them through the scalar cache, kUnroll degrees at a time.
constexpr int kPPTF = 4;
constexpr int kUnroll = 8;

__global__ void __launch_bounds__(64) k_rec_fwd(const ExecDesc* __restrict__ descs)
{
    const ExecDesc& d = descs[blockIdx.x];
    const int task = blockIdx.y;
    if (task >= d.ntasks) return;
    cptr<RecTask> tp = as_const(d.tasks) + task;
    const int p0 = uniform(tp->p0), np = uniform(tp->np), mode = uniform(tp->mode), cut = uniform(tp->cut);
    const int lane = threadIdx.x;
    const int64_t N = d.N;
    cptr<double> c = as_const(d.in);
    double res[kPPTF];
    if (mode == 0) {
        double x[kPPTF], u1[kPPTF], u2[kPPTF];
#pragma unroll
        for (int q = 0; q < kPPTF; ++q) {
            const int idx = lane + 64 * q;
            const int64_t i = p0 + (idx < np ? idx : 0);
            double s;
            sincospi((double)i / (double)N, &s, &x[q]);
            u1[q] = 0.0;
            u2[q] = 0.0;
        }
        cptr<d4> co = as_const(d.rec0);  // (A_n, B_n, C_{n+1})
        int n = cut - 1;
        for (; n >= kUnroll - 1; n -= kUnroll) {
            d4 qv[kUnroll];
            double cv[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                qv[k] = ld(co + (n - k));
                cv[k] = c[n - k];
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
#pragma unroll
                for (int q = 0; q < kPPTF; ++q) {
                    const double u0 = fma(fma(qv[k].x, x[q], qv[k].y), u1[q], fma(-qv[k].z, u2[q], cv[k]));
                    u2[q] = u1[q];
                    u1[q] = u0;
                }
            }
        }
        for (; n >= 0; --n) {
            const d4 qn = ld(co + n);
            const double cn = c[n];
#pragma unroll
            for (int q = 0; q < kPPTF; ++q) {
                const double u0 = fma(fma(qn.x, x[q], qn.y), u1[q], fma(-qn.z, u2[q], cn));
                u2[q] = u1[q];
                u1[q] = u0;
            }
        }
#pragma unroll
        for (int q = 0; q < kPPTF; ++q) res[q] = u1[q];
    } else {
        double dx[kPPTF], u[kPPTF], D[kPPTF];
#pragma unroll
        for (int q = 0; q < kPPTF; ++q) {
            const int idx = lane + 64 * q;
            const int64_t i = p0 + (idx < np ? idx : 0);
            double sh, ch;
            sincospi((double)i / (double)(2 * N), &sh, &ch);
            dx[q] = mode > 0 ? -2.0 * sh * sh : 2.0 * ch * ch;
            u[q] = 0.0;
            D[q] = 0.0;
        }
        cptr<d4> co = as_const(mode > 0 ? d.recp : d.recm);  // (A_n, C_{n+1} r_{n+1}, 1/r_n)
        int n = cut - 1;
        for (; n >= kUnroll; n -= kUnroll) {
            d4 qv[kUnroll];
            double cv[kUnroll];
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                qv[k] = ld(co + (n - k));
                cv[k] = c[n - k];
            }
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
#pragma unroll
                for (int q = 0; q < kPPTF; ++q) {
                    const double Dn = fma(qv[k].x * dx[q], u[q], fma(qv[k].y, D[q], cv[k]));
                    u[q] = fma(u[q], qv[k].z, Dn);
                    D[q] = Dn;
                }
            }
        }
        for (; n >= 1; --n) {
            const d4 qn = ld(co + n);
            const double cn = c[n];
#pragma unroll
            for (int q = 0; q < kPPTF; ++q) {
                const double Dn = fma(qn.x * dx[q], u[q], fma(qn.y, D[q], cn));
                u[q] = fma(u[q], qn.z, Dn);
                D[q] = Dn;
            }
        }
        if (cut >= 1) {
            const d4 qn = ld(co);
            const double cn = c[0];
#pragma unroll
            for (int q = 0; q < kPPTF; ++q) D[q] = fma(qn.x * dx[q], u[q], fma(qn.y, D[q], cn));
        }
#pragma unroll
        for (int q = 0; q < kPPTF; ++q) res[q] = D[q];
    }
#pragma unroll
    for (int q = 0; q < kPPTF; ++q) {
        const int idx = lane + 64 * q;
        if (idx < np) d.p[p0 + idx] = res[q];
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
    const ExecDesc& d = descs[blockIdx.x];
    const int task = blockIdx.y;
    if (task >= d.ntasks) return;
    cptr<RecTask> tp = as_const(d.tasks) + task;
    const int p0 = uniform(tp->p0), np = uniform(tp->np), mode = uniform(tp->mode), cut = uniform(tp->cut);
    const int64_t off = tp->off;
    const int lane = threadIdx.x;
    const int64_t G = d.G;
    double* __restrict__ part = d.part + off;

    double pv[kPPT], ev[kPPT], xv[kPPT];
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
        const int idx = lane + 64 * q;
        const bool act = idx < np;
        const int64_t j = p0 + (act ? idx : 0);
        const double g = act ? d.p[j] : 0.0;
        pv[q] = g;      // pi_0 = g_j (scaled recurrence)
        ev[q] = 0.0;    // e_0 = 0 (modified) / P_{-1} = 0 (three-term)
        if (mode == 0) {
            double s, x;
            sincospi((double)j / (double)G, &s, &x);
            xv[q] = x;
        } else {
            double sh, ch;
            sincospi((double)j / (double)(2 * G), &sh, &ch);
            xv[q] = mode > 0 ? -2.0 * sh * sh : 2.0 * ch * ch;
        }
    }
    cptr<d4> co = as_const(mode == 0 ? d.rec0 : (mode > 0 ? d.recp : d.recm));
    const int dd = lane >> 2, qq = lane & 3;  // reduction: degree dd of the chunk, quarter qq of the 64 lanes
    for (int n0 = 0; n0 < cut; n0 += kChunk) {
        const int nend = min(kChunk, cut - n0);
#pragma unroll 4
        for (int t = 0; t < nend; ++t) {
            const int n = n0 + t;
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < kPPT; ++q) v += pv[q];
            red[t][lane] = v;
            const d4 cf = ld(co + n);
            if (mode == 0) {
                // rec0 holds (A_n, B_n, C_n) for the three-term recurrence
#pragma unroll
                for (int q = 0; q < kPPT; ++q) {
                    const double p1 = fma(fma(cf.x, xv[q], cf.y), pv[q], -cf.z * ev[q]);
                    ev[q] = pv[q];
                    pv[q] = p1;
                }
            } else {
                // (A_n, C_n / r_{n-1}, r_n)
#pragma unroll
                for (int q = 0; q < kPPT; ++q) {
                    const double e1 = fma(cf.x * xv[q], pv[q], cf.y * ev[q]);
                    pv[q] = fma(pv[q], cf.z, e1);
                    ev[q] = e1;
                }
            }
        }
        __syncthreads();
        if (dd < nend) {
            double s = 0.0;
#pragma unroll
            for (int l = 0; l < 16; ++l) s += red[dd][qq * 16 + l];
            s += __shfl_xor(s, 1);
            s += __shfl_xor(s, 2);
            if (qq == 0) part[n0 + dd] = s;
        }
        __syncthreads();
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
