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

__global__ void __launch_bounds__(64) k_rec_fwd(const ExecDesc* __restrict__ descs)
{
    const ExecDesc& d = descs[blockIdx.x];
    const int task = blockIdx.y;
    if (task >= d.ntasks) return;
    const RecTask tk = d.tasks[task];
    const int lane = threadIdx.x;
    const bool active = lane < tk.np;
    const int64_t i = tk.p0 + (active ? lane : 0);
    const int64_t N = d.N;
    const double* __restrict__ c = d.in;
    const int cut = tk.cut;
    double res = 0.0;
    if (tk.mode == 0) {
        double s, x;
        sincospi((double)i / (double)N, &s, &x);
        const double4* __restrict__ co = d.rec0;  // (A_n, B_n, C_{n+1})
        double u1 = 0.0, u2 = 0.0;
        for (int n = cut - 1; n >= 0; --n) {
            const double4 q = co[n];
            const double u0 = fma(fma(q.x, x, q.y), u1, fma(-q.z, u2, c[n]));
            u2 = u1;
            u1 = u0;
        }
        res = u1;
    } else {
        double sh, ch;
        sincospi((double)i / (double)(2 * N), &sh, &ch);
        const double dx = tk.mode > 0 ? -2.0 * sh * sh : 2.0 * ch * ch;
        const double4* __restrict__ co = tk.mode > 0 ? d.recp : d.recm;  // (A_n, C_{n+1} r_{n+1}, 1/r_n)
        double u = 0.0, D = 0.0;
        for (int n = cut - 1; n >= 1; --n) {
            const double4 q = co[n];
            const double Dn = fma(q.x * dx, u, fma(q.y, D, c[n]));
            u = fma(u, q.z, Dn);
            D = Dn;
        }
        if (cut >= 1) {
            const double4 q = co[0];
            D = fma(q.x * dx, u, fma(q.y, D, c[0]));
        }
        res = D;
    }
    if (active) d.p[i] = res;
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
    const RecTask tk = d.tasks[task];
    const int lane = threadIdx.x;
    const int64_t G = d.G;
    const int cut = tk.cut;
    double* __restrict__ part = d.part + tk.off;

    double pv[kPPT], ev[kPPT], xv[kPPT];
#pragma unroll
    for (int q = 0; q < kPPT; ++q) {
        const int idx = lane + 64 * q;
        const bool act = idx < tk.np;
        const int64_t j = tk.p0 + (act ? idx : 0);
        const double g = act ? d.p[j] : 0.0;
        pv[q] = g;      // pi_0 = g_j (scaled recurrence)
        ev[q] = 0.0;    // e_0 = 0 (modified) / P_{-1} = 0 (three-term)
        if (tk.mode == 0) {
            double s, x;
            sincospi((double)j / (double)G, &s, &x);
            xv[q] = x;
        } else {
            double sh, ch;
            sincospi((double)j / (double)(2 * G), &sh, &ch);
            xv[q] = tk.mode > 0 ? -2.0 * sh * sh : 2.0 * ch * ch;
        }
    }
    const double4* __restrict__ co = tk.mode == 0 ? d.rec0 : (tk.mode > 0 ? d.recp : d.recm);
    const int dd = lane >> 2, qq = lane & 3;  // reduction: degree dd of the chunk, quarter qq of the 64 lanes
    for (int n0 = 0; n0 < cut; n0 += kChunk) {
        const int nend = min(kChunk, cut - n0);
        for (int t = 0; t < nend; ++t) {
            const int n = n0 + t;
            double v = 0.0;
#pragma unroll
            for (int q = 0; q < kPPT; ++q) v += pv[q];
            red[t][lane] = v;
            const double4 cf = co[n];
            if (tk.mode == 0) {
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
    for (int t = 0; t < d.ntasks; ++t) {
        const RecTask tk = d.tasks[t];
        if (tk.cut <= n) break;
        acc += d.part[tk.off + n];
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
