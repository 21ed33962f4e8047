// Real-input DFTs behind every DCT-I / DST-I of the transform.
//
// All of them have the form
//     X_s = sum_{q < 2L} r_q exp(+i pi q s / L),   s = 0..L,   r real,
// computed from one complex FFT of length L on z_t = r_{2t} + i r_{2t+1}
// followed by the standard untangling
//     X_s = E_s + e^{i pi s/L} O_s,   E_s = (Z_s + conj Z_{L-s})/2,   O_s = (Z_s - conj Z_{L-s})/(2i).
// Re X is a DCT-I and Im X a DST-I of the same data (Sec. 2.1: T_N is a
// diagonally scaled DCT-I, the sine matrix a DST-I bordered by zeros).
//
// What r is and what happens to X is set by a source and a sink:
//   FwdAsy  / FwdAsy : the Hahn blocks of the forward transform (eq. PNASY):
//                      r_n = C_{n,m} c_n on the block's degrees, and
//                      p_i += u_m(theta_i) Re X_i + v_m(theta_i) Im X_i on its window;
//   InvAsy  / InvAsy : the transposed blocks of the inverse (Sec. 3.2): r built
//                      from a_j = u_m g_j, b_j = v_m g_j on the window so that
//                      Re X_n + Im X_n = sum_j a_j cos(pi n j/2N) + b_j sin(pi n j/2N),
//                      and y_n = sum_m C_{n,m} (...) on the block's degrees;
//   FwdFinal/ FwdFinal: c_cheb = T_N^{-1} p (diagonally scaled DCT-I);
//   InvInit / InvInit : g_j = w_j f_j with f = T_{2N}^T [c_cheb; 0] (eq. CJTT);
//   Moments / Weights : Clenshaw--Curtis weights from modified moments (eq. CCweights).
//
// Lengths up to kSingleMax run in one workgroup (whole transform in LDS);
// longer ones in two passes L = L1 * L2: a column pass (L1-point FFTs over
// stride L2, times exp(2 pi i n2 k1 / L)) writes intermediates to global memory,
// and a row pass (L2-point FFTs) pairs rows k1 and L1-k1 so each workgroup has
// both Z_s and Z_{L-s} for the untangling.  The row pass loops over all Hahn
// terms (m) and blocks (k) of its rows and accumulates in registers, so each
// output is written once.
#include <algorithm>

#include "cjt_internal.h"
#include "fft_lds.h"

namespace cjt {

// ------------------------------------------------------------------ sources

template <Src S>
struct Source;

template <>
struct Source<Src::FwdAsy> {
    // job = k * M + m
    __device__ static bool valid(const ExecDesc& d, int job) { return job < d.nblk * d.M; }
    __device__ static cx<double> load(const ExecDesc& d, int job, int64_t t)
    {
        const int k = job / d.M, m = job - k * d.M;
        const int64_t lo = d.deg_lo[k], hi = d.deg_hi[k];
        const int64_t n0 = 2 * t, n1 = n0 + 1;
        const double* Cm = d.C + (int64_t)m * (d.N + 1);
        double x0 = (n0 >= lo && n0 < hi) ? Cm[n0] * d.in[n0] : 0.0;
        double x1 = (n1 >= lo && n1 < hi) ? Cm[n1] * d.in[n1] : 0.0;
        return {x0, x1};
    }
};

template <>
struct Source<Src::InvAsy> {
    __device__ static bool valid(const ExecDesc& d, int job) { return job < d.nblk * d.M; }
    // a_j = u_m(theta_j) g_j, b_j = v_m(theta_j) g_j on the window (zero elsewhere);
    // r_0 = a_0, r_G = a_G, r_j = (a_j + b_j)/2 and r_{2G-j} = (a_j - b_j)/2 for 0 < j < G.
    __device__ static double r(const ExecDesc& d, int k, const cx<double>* uvm, int64_t q)
    {
        const int64_t G = d.G;
        int64_t j;
        double sb;
        if (q <= G) { j = q; sb = 1.0; }
        else { j = 2 * G - q; sb = -1.0; }
        if (j < d.win_lo[k] || j > d.win_hi[k]) return 0.0;
        const double g = d.p[j];
        const cx<double> uv = uvm[j];
        if (j == 0 || j == G) return uv.re * g;
        return 0.5 * (uv.re * g + sb * uv.im * g);
    }
    __device__ static cx<double> load(const ExecDesc& d, int job, int64_t t)
    {
        const int k = job / d.M, m = job - k * d.M;
        const cx<double>* uvm = d.uv + (int64_t)m * (d.G + 1);
        return {r(d, k, uvm, 2 * t), r(d, k, uvm, 2 * t + 1)};
    }
};

template <>
struct Source<Src::FwdFinal> {
    __device__ static bool valid(const ExecDesc&, int job) { return job == 0; }
    // p = recurrence part + Hahn-block part (the latter only if the plan has blocks)
    __device__ static double pv(const ExecDesc& d, int64_t j) { return d.nblk > 0 ? d.p[j] + d.p2[j] : d.p[j]; }
    __device__ static cx<double> load(const ExecDesc& d, int, int64_t t)
    {
        const int64_t N = d.N, j0 = 2 * t, j1 = j0 + 1;
        double x0 = j0 <= N ? pv(d, j0) * ((j0 == 0 || j0 == N) ? 0.5 : 1.0) : 0.0;
        double x1 = j1 <= N ? pv(d, j1) * ((j1 == N) ? 0.5 : 1.0) : 0.0;
        return {x0, x1};
    }
};

template <>
struct Source<Src::InvInit> {
    __device__ static bool valid(const ExecDesc&, int job) { return job == 0; }
    __device__ static cx<double> load(const ExecDesc& d, int, int64_t t)
    {
        const int64_t N = d.N, k0 = 2 * t, k1 = k0 + 1;
        return {k0 <= N ? d.in[k0] : 0.0, k1 <= N ? d.in[k1] : 0.0};
    }
};

template <>
struct Source<Src::Moments> {
    // in = mu_0..mu_G, halved at both ends
    __device__ static bool valid(const ExecDesc&, int job) { return job == 0; }
    __device__ static cx<double> load(const ExecDesc& d, int, int64_t t)
    {
        const int64_t G = d.G, k0 = 2 * t, k1 = k0 + 1;
        double x0 = k0 <= G ? d.in[k0] * ((k0 == 0 || k0 == G) ? 0.5 : 1.0) : 0.0;
        double x1 = k1 <= G ? d.in[k1] * ((k1 == G) ? 0.5 : 1.0) : 0.0;
        return {x0, x1};
    }
};

// ------------------------------------------------------------------ sinks
// contrib() sees every output index s in [0, L] exactly once per job and
// returns what that job adds to output s; finish() stores the sum over jobs.

constexpr int kSlots = 20;
constexpr int kEPT = 8;  // row-pass elements per thread: 2048 per 256-thread workgroup

template <Sink S>
struct Target;

template <>
struct Target<Sink::FwdAsy> {
    __device__ static double contrib(const ExecDesc& d, int job, int64_t i, cx<double> X)
    {
        const int k = job / d.M, m = job - k * d.M;
        if (i < d.win_lo[k] || i > d.win_hi[k]) return 0.0;
        const cx<double> uv = d.uv[(int64_t)m * (d.G + 1) + i];
        return fma(uv.re, X.re, uv.im * X.im);
    }
    // every point is written (zero outside the windows); the final DCT-I adds
    // the recurrence part
    __device__ static void finish(const ExecDesc& d, int64_t i, double v) { d.p2[i] = v; }
};

template <>
struct Target<Sink::InvAsy> {
    __device__ static double contrib(const ExecDesc& d, int job, int64_t n, cx<double> X)
    {
        const int k = job / d.M, m = job - k * d.M;
        if (n < d.deg_lo[k] || n >= d.deg_hi[k]) return 0.0;
        return d.C[(int64_t)m * (d.N + 1) + n] * (X.re + X.im);
    }
    // Every degree 0..N is written (zero outside the blocks); the recurrence
    // reduction adds its part and applies 1/A_n afterwards.
    __device__ static void finish(const ExecDesc& d, int64_t n, double v)
    {
        if (n <= d.N) d.out[n] = v;
    }
};

template <>
struct Target<Sink::FwdFinal> {
    __device__ static double contrib(const ExecDesc&, int, int64_t, cx<double> X) { return X.re; }
    __device__ static void finish(const ExecDesc& d, int64_t k, double v)
    {
        const int64_t N = d.N;
        const double sc = (k == 0 || k == N) ? 1.0 / (double)N : 2.0 / (double)N;
        d.out[k] = sc * v;
    }
};

template <>
struct Target<Sink::InvInit> {
    __device__ static double contrib(const ExecDesc&, int, int64_t, cx<double> X) { return X.re; }
    __device__ static void finish(const ExecDesc& d, int64_t j, double v) { d.p[j] = d.w[j] * v; }
};

template <>
struct Target<Sink::Weights> {
    __device__ static double contrib(const ExecDesc&, int, int64_t, cx<double> X) { return X.re; }
    // w_j = (1 - (d_j0 + d_jG)/2) / (G/2) Re X_j
    __device__ static void finish(const ExecDesc& d, int64_t j, double v)
    {
        const int64_t G = d.G;
        const double sc = ((j == 0 || j == G) ? 0.5 : 1.0) / (0.5 * (double)G);
        d.out[j] = sc * v;
    }
};

// ------------------------------------------------------------------ untangling

template <typename T>
struct Untangled {
    cx<double> xa, xb;  // X_s and X_{L-s}
};

// From Z_s, Z_{L-s} (s not 0, not L/2): X_s = E + W O, X_{L-s} = conj(E - W O), W = tw[s].
template <typename T>
__device__ __forceinline__ void untangle(cx<T> za, cx<T> zb, cx<T> w, cx<double>& xs, cx<double>& xls)
{
    cx<T> zbc = conj(zb);
    cx<T> e = {(T)0.5 * (za.re + zbc.re), (T)0.5 * (za.im + zbc.im)};
    cx<T> dd = {(T)0.5 * (za.re - zbc.re), (T)0.5 * (za.im - zbc.im)};
    cx<T> o = cmul_mi(dd);  // (za - conj zb) / (2i)
    cx<T> wo = cmul(w, o);
    xs = {(double)(e.re + wo.re), (double)(e.im + wo.im)};
    xls = {(double)(e.re - wo.re), -(double)(e.im - wo.im)};
}

// ------------------------------------------------------------------ single pass

template <typename T>
__device__ __forceinline__ cx<T> to_t(cx<double> v) { return {(T)v.re, (T)v.im}; }

// One workgroup per instance; the whole length-L transform lives in LDS.
// Loops over all jobs of the instance and accumulates per thread.
template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_single(const ExecDesc* __restrict__ descs, FftGeom g, int max_jobs,
                                                size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[blockIdx.x];
    const int L = (int)g.L;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const int nel = L / 2 + 1;  // elements s = 0..L/2
    // per-thread accumulators in LDS: acc[slot * nth + tid]
    double* acc = reinterpret_cast<double*>(smem_raw + acc_off);
    for (int i = 0; i < kSlots; ++i) acc[i * nth + tid] = 0.0;

    for (int job = 0; job < max_jobs; ++job) {
        if (!Source<S>::valid(d, job)) break;
        for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = to_t<T>(Source<S>::load(d, job, t));
        __syncthreads();
        lds_fft<T>(buf, g.logL, 1, tw, 2 * g.L);
#pragma unroll 2
        for (int q = 0; q < kSlots / 2; ++q) {
            const int s = tid + q * nth;
            if (s >= nel) break;
            cx<double> xa, xb;
            if (s == 0) {
                cx<T> z = buf[lds_pad(0)];
                xa = {(double)z.re + (double)z.im, 0.0};
                xb = {(double)z.re - (double)z.im, 0.0};
            } else if (2 * s == L) {
                cx<T> z = buf[lds_pad(s)];
                xa = {(double)z.re, (double)z.im};
                xb = xa;
            } else {
                untangle<T>(buf[lds_pad(s)], buf[lds_pad(L - s)], tw[s], xa, xb);
            }
            acc[(2 * q) * nth + tid] += Target<K>::contrib(d, job, s, xa);
            if (2 * s != L) acc[(2 * q + 1) * nth + tid] += Target<K>::contrib(d, job, L - s, xb);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kSlots / 2; ++q) {
        const int s = tid + q * nth;
        if (s >= nel) break;
        Target<K>::finish(d, s, acc[(2 * q) * nth + tid]);
        if (2 * s != L) Target<K>::finish(d, L - s, acc[(2 * q + 1) * nth + tid]);
    }
}

// ------------------------------------------------------------------ two passes

// Column pass: TC consecutive columns n2 per workgroup, L1-point FFTs over n1
// held in registers (thread lt of a column owns n1 = lt + r L1/16), multiplied
// by exp(2 pi i n2 k1 / L) and written to tmp[job][k1 L2 + n2].
template <typename T, Src S>
__global__ void __launch_bounds__(256) k_pass1(const ExecDesc* __restrict__ descs, FftGeom g, int TC)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[blockIdx.z];
    const int job = blockIdx.y;
    if (!Source<S>::valid(d, job)) return;
    const int L1 = g.L1, L2 = g.L2;
    const int64_t L = g.L;
    const int tid = threadIdx.x;
    const int c = tid % TC, lt = tid / TC;
    const int64_t col = (int64_t)blockIdx.x * TC + c;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const int step = L1 >> 4;
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = to_t<T>(Source<S>::load(d, job, (int64_t)(lt + r * step) * L2 + col));
    fft_reg<T>(v, lds + c * slice_stride(L1), g.logL1, lt, true, tw, 2 * L);
    cx<T>* out = reinterpret_cast<cx<T>*>(d.tmp) + (int64_t)job * L;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int64_t k1 = fft_out_index(s, lt, g.logL1);
        const int64_t q = (2 * col * k1) & (2 * L - 1);  // exp(2 pi i n2 k1 / L) = tw[2 n2 k1 mod 2L]
        out[k1 * L2 + col] = cmul(v[s], tw[q]);
    }
}

// Row pass: TU units per workgroup; unit u holds rows u and L1-u (unit 0 holds
// rows 0 and L1/2).  Element (u, k2) pairs Z at row u, position k2 with Z at
// row L1-u, position L2-1-k2, which are Z_s and Z_{L-s} for s = u + L1 k2.
// The L2-point FFTs run in registers; their outputs go through LDS once so
// that each thread can fetch both members of its pairs.
template <typename T, Sink K>
__global__ void __launch_bounds__(256) k_pass2(const ExecDesc* __restrict__ descs, FftGeom g, int TU, int max_jobs,
                                               int src_single_job, size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[blockIdx.z];
    const int L1 = g.L1, L2 = g.L2;
    const int64_t L = g.L;
    const int unit0 = blockIdx.x * TU;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const int tpr = L2 >> 4;               // threads per row
    const int rs = tid / tpr, lt = tid - rs * tpr;
    const int my_unit = unit0 + (rs >> 1);
    const int my_row = (rs & 1) == 0 ? my_unit : (my_unit == 0 ? L1 / 2 : L1 - my_unit);
    // TU * L2 regular elements per workgroup, kEPT = 8 per thread (nth = TU L2 / 8)
    constexpr int ept = kEPT;
    const bool has_half = (unit0 == 0) && (tid == nth - 1);  // thread that also owns s = L/2

    // per-thread accumulators in LDS: acc[slot * nth + tid], slots 0..2*ept (2*ept = s = L/2)
    double* acc = reinterpret_cast<double*>(smem_raw + acc_off);
    for (int i = 0; i <= 2 * ept; ++i) acc[i * nth + tid] = 0.0;

    // jobs in the order (m, k), k fastest, so that the diagonals of term m are
    // re-read from L2 for every block
    const int njobs = src_single_job ? 1 : d.nblk * d.M;
    for (int it = 0; it < njobs; ++it) {
        const int job = src_single_job ? 0 : (it % d.nblk) * d.M + it / d.nblk;
        const cx<T>* in = reinterpret_cast<const cx<T>*>(d.tmp) + (int64_t)job * L + (int64_t)my_row * L2;
        cx<T> v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = in[lt + r * tpr];
        cx<T>* slice = buf + rs * slice_stride(L2);
        fft_reg<T>(v, slice, g.logL2, lt, true, tw, 2 * L);
#pragma unroll
        for (int s = 0; s < 16; ++s) slice[lds_pad(fft_out_index(s, lt, g.logL2))] = v[s];
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < ept; ++q) {
            const int eps = tid + q * nth;
            const int lu = eps % TU, k2 = eps / TU;
            const int unit = unit0 + lu;
            const int ra = 2 * lu, rb = 2 * lu + 1;
            cx<double> xa, xb;
            int64_t s;
            if (unit == 0) {
                if (k2 < L2 / 2) {
                    s = L1 / 2 + (int64_t)L1 * k2;
                    untangle<T>(buf[rb * slice_stride(L2) + lds_pad(k2)], buf[rb * slice_stride(L2) + lds_pad(L2 - 1 - k2)], tw[s], xa, xb);
                } else if (k2 == L2 / 2) {
                    s = 0;
                    cx<T> z = buf[ra * slice_stride(L2)];
                    xa = {(double)z.re + (double)z.im, 0.0};
                    xb = {(double)z.re - (double)z.im, 0.0};
                } else {
                    const int kk = k2 - L2 / 2;
                    s = (int64_t)L1 * kk;
                    untangle<T>(buf[ra * slice_stride(L2) + lds_pad(kk)], buf[ra * slice_stride(L2) + lds_pad(L2 - kk)], tw[s], xa, xb);
                }
            } else {
                s = unit + (int64_t)L1 * k2;
                untangle<T>(buf[ra * slice_stride(L2) + lds_pad(k2)], buf[rb * slice_stride(L2) + lds_pad(L2 - 1 - k2)], tw[s], xa, xb);
            }
            acc[(2 * q) * nth + tid] += Target<K>::contrib(d, job, s, xa);
            acc[(2 * q + 1) * nth + tid] += Target<K>::contrib(d, job, L - s, xb);
        }
        if (has_half) {
            cx<T> z = buf[lds_pad(L2 / 2)];  // row 0, position L2/2: s = L/2
            acc[(2 * ept) * nth + tid] += Target<K>::contrib(d, job, L / 2, cx<double>{(double)z.re, (double)z.im});
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < ept; ++q) {
        const int eps = tid + q * nth;
        const int lu = eps % TU, k2 = eps / TU;
        const int unit = unit0 + lu;
        int64_t s;
        if (unit == 0) {
            if (k2 < L2 / 2) s = L1 / 2 + (int64_t)L1 * k2;
            else if (k2 == L2 / 2) s = 0;
            else s = (int64_t)L1 * (k2 - L2 / 2);
        } else {
            s = unit + (int64_t)L1 * k2;
        }
        Target<K>::finish(d, s, acc[(2 * q) * nth + tid]);
        Target<K>::finish(d, L - s, acc[(2 * q + 1) * nth + tid]);
    }
    if (has_half) Target<K>::finish(d, L / 2, acc[(2 * ept) * nth + tid]);
}

// ------------------------------------------------------------------ chirp-z (any L)
//
// For L not a power of two the length-L complex FFT Z_s = sum_t z_t e^{2 pi i ts/L}
// uses ts = (t^2 + s^2 - (s-t)^2)/2:  Z_s = c_s (a * b)_s with a_t = z_t c_t,
// c_t = e^{i pi t^2/L}, b_k = conj(c_|k|), and the linear convolution is a cyclic
// one of length P >= 2L-1:  a * b = F^-1(F(a) F(b~)),  F^-1(X) = conj(F(conj X))/P.
// F(b~) is a per-length table.  Per job: two P-point transforms (column + row
// passes each), then the untangling of the length-2L real DFT from Z.
//
// Job storage (complex, per job): [0, P) column-pass output, [P, 2P) first
// transform in natural order, [2P, 2P+L) Z.

template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// stage 0: kernel spectrum (input b~ from the chirp table, output to bl)
// stage 1: input a_t = source(t) c_t, output A (natural order)
// stage 2: input conj(A_t F(b~)_t), output Z_s = c_s conj(E_s)/P for s < L
template <typename T, Src S, int STAGE>
__global__ void __launch_bounds__(256) k_bs_col(const ExecDesc* __restrict__ descs, FftGeom g, int TC, cx<T>* scratch)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int64_t P = g.P, L = g.L;
    const int P1 = g.L1, P2 = g.L2;
    const int job = blockIdx.y;
    const ExecDesc* d = STAGE == 0 ? nullptr : &descs[blockIdx.z];
    if constexpr (STAGE != 0)
        if (!Source<S>::valid(*d, job)) return;
    const int tid = threadIdx.x;
    const int c = tid % TC, lt = tid / TC;
    const int64_t col = (int64_t)blockIdx.x * TC + c;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    const cx<T>* bl = reinterpret_cast<const cx<T>*>(g.bl);
    cx<T>* base = STAGE == 0 ? scratch : reinterpret_cast<cx<T>*>(d->tmp) + (int64_t)job * (2 * P + L);
    const int step = P1 >> 4;
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t t = (int64_t)(lt + r * step) * P2 + col;
        cx<T> x = {(T)0, (T)0};
        if constexpr (STAGE == 0) {
            if (t < L) x = conj(chirp[t]);
            else if (t > P - L) x = conj(chirp[P - t]);
        } else if constexpr (STAGE == 1) {
            if (t < L) x = cmul(to_t<T>(Source<S>::load(*d, job, t)), chirp[t]);
        } else {
            x = conj(cmul(base[P + t], bl[t]));
        }
        v[r] = x;
    }
    fft_reg<T>(v, lds + c * slice_stride(P1), g.logL1, lt, true, tw, 2 * P);
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
        const int64_t k1 = fft_out_index(s2, lt, g.logL1);
        const int64_t q = (2 * col * k1) & (2 * P - 1);
        base[k1 * P2 + col] = cmul(v[s2], tw[q]);
    }
}

template <typename T, Src S, int STAGE>
__global__ void __launch_bounds__(256) k_bs_row(const ExecDesc* __restrict__ descs, FftGeom g, int TR, cx<T>* scratch,
                                                cx<T>* bl_out)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const int64_t P = g.P, L = g.L;
    const int P1 = g.L1, P2 = g.L2;
    const int job = blockIdx.y;
    const ExecDesc* d = STAGE == 0 ? nullptr : &descs[blockIdx.z];
    if constexpr (STAGE != 0)
        if (!Source<S>::valid(*d, job)) return;
    const int tid = threadIdx.x;
    const int tpr = P2 >> 4;
    const int rr = tid / tpr, lt = tid - rr * tpr;
    const int64_t k1 = (int64_t)blockIdx.x * TR + rr;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    cx<T>* base = STAGE == 0 ? scratch : reinterpret_cast<cx<T>*>(d->tmp) + (int64_t)job * (2 * P + L);
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = base[k1 * P2 + lt + r * tpr];
    fft_reg<T>(v, lds + rr * slice_stride(P2), g.logL2, lt, true, tw, 2 * P);
    const T invP = (T)1 / (T)P;
#pragma unroll
    for (int s2 = 0; s2 < 16; ++s2) {
        const int64_t k2 = fft_out_index(s2, lt, g.logL2);
        const int64_t sidx = k1 + (int64_t)P1 * k2;
        if constexpr (STAGE == 0) bl_out[sidx] = v[s2];
        else if constexpr (STAGE == 1) base[P + sidx] = v[s2];
        else if (sidx < L) base[2 * P + sidx] = cmul(chirp[sidx], cscale(conj(v[s2]), invP));
    }
}

// Untangling of the length-2L real DFT from Z, summed over the jobs of the
// instance (terms m outer, blocks k inner); one element (s, L-s) per thread.
template <typename T, Sink K>
__global__ void __launch_bounds__(256) k_bs_untangle(const ExecDesc* __restrict__ descs, FftGeom g, int single_job)
{
    const ExecDesc& d = descs[blockIdx.y];
    const int64_t L = g.L, P = g.P;
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s > L / 2) return;
    const cx<T>* utw = reinterpret_cast<const cx<T>*>(g.utw);
    const int njobs = single_job ? 1 : d.nblk * d.M;
    double a0 = 0.0, a1 = 0.0;
    for (int it = 0; it < njobs; ++it) {
        const int job = single_job ? 0 : (it % d.nblk) * d.M + it / d.nblk;
        const cx<T>* Z = reinterpret_cast<const cx<T>*>(d.tmp) + (int64_t)job * (2 * P + L) + 2 * P;
        cx<double> xa, xb;
        if (s == 0) {
            const cx<T> z = Z[0];
            xa = {(double)z.re + (double)z.im, 0.0};
            xb = {(double)z.re - (double)z.im, 0.0};
        } else if (2 * s == L) {
            const cx<T> z = Z[s];
            xa = {(double)z.re, (double)z.im};
            xb = xa;
        } else {
            untangle<T>(Z[s], Z[L - s], utw[s], xa, xb);
        }
        a0 += Target<K>::contrib(d, job, s, xa);
        if (2 * s != L) a1 += Target<K>::contrib(d, job, L - s, xb);
    }
    Target<K>::finish(d, s, a0);
    if (2 * s != L) Target<K>::finish(d, L - s, a1);
}

// Whole chirp-z transform in one workgroup (P <= kSingleMax), looping over the jobs.
template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_bs_single(const ExecDesc* __restrict__ descs, FftGeom g, int max_jobs,
                                                   size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[blockIdx.x];
    const int L = (int)g.L, P = (int)g.P;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    const cx<T>* bl = reinterpret_cast<const cx<T>*>(g.bl);
    const cx<T>* utw = reinterpret_cast<const cx<T>*>(g.utw);
    const int nel = L / 2 + 1;
    double* acc = reinterpret_cast<double*>(smem_raw + acc_off);
    for (int i = 0; i < kSlots; ++i) acc[i * nth + tid] = 0.0;
    const T invP = (T)1 / (T)P;
    for (int job = 0; job < max_jobs; ++job) {
        if (!Source<S>::valid(d, job)) break;
        for (int t = tid; t < P; t += nth)
            buf[lds_pad(t)] = t < L ? cmul(to_t<T>(Source<S>::load(d, job, t)), chirp[t]) : cx<T>{(T)0, (T)0};
        __syncthreads();
        lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
        for (int t = tid; t < P; t += nth) buf[lds_pad(t)] = conj(cmul(buf[lds_pad(t)], bl[t]));
        __syncthreads();
        lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
        for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = cmul(chirp[t], cscale(conj(buf[lds_pad(t)]), invP));
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < kSlots / 2; ++q) {
            const int sx = tid + q * nth;
            if (sx >= nel) break;
            cx<double> xa, xb;
            if (sx == 0) {
                cx<T> z = buf[lds_pad(0)];
                xa = {(double)z.re + (double)z.im, 0.0};
                xb = {(double)z.re - (double)z.im, 0.0};
            } else if (2 * sx == L) {
                cx<T> z = buf[lds_pad(sx)];
                xa = {(double)z.re, (double)z.im};
                xb = xa;
            } else {
                untangle<T>(buf[lds_pad(sx)], buf[lds_pad(L - sx)], utw[sx], xa, xb);
            }
            acc[(2 * q) * nth + tid] += Target<K>::contrib(d, job, sx, xa);
            if (2 * sx != L) acc[(2 * q + 1) * nth + tid] += Target<K>::contrib(d, job, L - sx, xb);
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kSlots / 2; ++q) {
        const int sx = tid + q * nth;
        if (sx >= nel) break;
        Target<K>::finish(d, sx, acc[(2 * q) * nth + tid]);
        if (2 * sx != L) Target<K>::finish(d, L - sx, acc[(2 * q + 1) * nth + tid]);
    }
}

// ------------------------------------------------------------------ launch

namespace {

size_t lds_bytes(int n_elems, size_t esz) { return (size_t)(n_elems + (n_elems >> 4) + 1) * esz; }

// Workgroups of this engine use up to ~70 KB of LDS (gfx950 has 160 KB per CU);
// raise the dynamic-LDS limit of each kernel once before its first launch.
template <typename K>
cjt_status allow_lds(K kernel, size_t bytes)
{
    CJT_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    return CJT_OK;
}

template <typename T, Src S, Sink K>
cjt_status run_bs(const EngineArgs& a, int max_jobs, bool single_job)
{
    const FftGeom& g = a.geom;
    const size_t esz = sizeof(cx<T>);
    if (g.single) {
        const int P = (int)g.P;
        int nth = P / 16;
        if (nth < 64) nth = 64;
        if (nth > 256) nth = 256;
        if (((int)g.L / 2 + 1 + nth - 1) / nth > kSlots / 2) return fail(CJT_EUNSUPPORTED, "chirp-z length too large");
        const size_t acc_off = (lds_bytes(P, esz) + 255) & ~(size_t)255;
        const size_t total = acc_off + sizeof(double) * kSlots * nth;
        cjt_status st = allow_lds(k_bs_single<T, S, K>, total);
        if (st != CJT_OK) return st;
        ProfScope ps(a.name1, a.flops1 + a.flops2, a.bytes1 + a.bytes2, a.stream);
        hipLaunchKernelGGL((k_bs_single<T, S, K>), dim3(a.count), dim3(nth), total, a.stream, a.d_desc, g, max_jobs,
                           acc_off);
        CJT_HIP_TRY(hipGetLastError());
        return CJT_OK;
    }
    const int TC = std::max(1, 2048 / g.L1);
    const int TR = std::max(1, 2048 / g.L2);
    const int nth1 = TC * (g.L1 / 16), nth2 = TR * (g.L2 / 16);
    if (g.L2 % TC != 0 || g.L1 % TR != 0 || nth1 > 256 || nth2 > 256) return fail(CJT_EUNSUPPORTED, "chirp-z split");
    const size_t lds1 = (size_t)TC * slice_stride(g.L1) * esz, lds2 = (size_t)TR * slice_stride(g.L2) * esz;
    cjt_status st = allow_lds(k_bs_col<T, S, 1>, lds1);
    if (st == CJT_OK) st = allow_lds(k_bs_col<T, S, 2>, lds1);
    if (st == CJT_OK) st = allow_lds(k_bs_row<T, S, 1>, lds2);
    if (st == CJT_OK) st = allow_lds(k_bs_row<T, S, 2>, lds2);
    if (st != CJT_OK) return st;
    const dim3 gc(g.L2 / TC, max_jobs, a.count), gr(g.L1 / TR, max_jobs, a.count);
    {
        ProfScope ps(a.name1, 0.5 * a.flops1, 0.5 * a.bytes1, a.stream);
        hipLaunchKernelGGL((k_bs_col<T, S, 1>), gc, dim3(nth1), lds1, a.stream, a.d_desc, g, TC, (cx<T>*)nullptr);
        CJT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_bs_row<T, S, 1>), gr, dim3(nth2), lds2, a.stream, a.d_desc, g, TR, (cx<T>*)nullptr,
                           (cx<T>*)nullptr);
        CJT_HIP_TRY(hipGetLastError());
    }
    {
        ProfScope ps(a.name1, 0.5 * a.flops1, 0.5 * a.bytes1, a.stream);
        hipLaunchKernelGGL((k_bs_col<T, S, 2>), gc, dim3(nth1), lds1, a.stream, a.d_desc, g, TC, (cx<T>*)nullptr);
        CJT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_bs_row<T, S, 2>), gr, dim3(nth2), lds2, a.stream, a.d_desc, g, TR, (cx<T>*)nullptr,
                           (cx<T>*)nullptr);
        CJT_HIP_TRY(hipGetLastError());
    }
    {
        ProfScope ps(a.name2, a.flops2, a.bytes2, a.stream);
        const dim3 gu((unsigned)((g.L / 2 + 1 + 255) / 256), a.count);
        hipLaunchKernelGGL((k_bs_untangle<T, K>), gu, dim3(256), 0, a.stream, a.d_desc, g, single_job ? 1 : 0);
        CJT_HIP_TRY(hipGetLastError());
    }
    return CJT_OK;
}

template <typename T, Src S, Sink K>
cjt_status run(const EngineArgs& a)
{
    const FftGeom& g = a.geom;
    const size_t esz = sizeof(cx<T>);
    const bool single_job = (S != Src::FwdAsy && S != Src::InvAsy);
    const int max_jobs = single_job ? 1 : a.max_jobs;
    if (max_jobs <= 0 || a.count <= 0) return CJT_OK;
    if (g.bluestein) return run_bs<T, S, K>(a, max_jobs, single_job);
    if (g.single) {
        const int L = (int)g.L;
        int nth = L / 16;
        if (nth < 64) nth = 64;
        if (nth > 256) nth = 256;
        if ((L / 2 + 1 + nth - 1) / nth > kSlots / 2) return fail(CJT_EUNSUPPORTED, "single-pass length too large");
        const size_t acc_off = (lds_bytes(L, esz) + 255) & ~(size_t)255;
        const size_t total = acc_off + sizeof(double) * kSlots * nth;
        cjt_status st = allow_lds(k_single<T, S, K>, total);
        if (st != CJT_OK) return st;
        ProfScope ps(a.name1, a.flops1 + a.flops2, a.bytes1 + a.bytes2, a.stream);
        hipLaunchKernelGGL((k_single<T, S, K>), dim3(a.count), dim3(nth), total, a.stream, a.d_desc, g, max_jobs,
                           acc_off);
        CJT_HIP_TRY(hipGetLastError());
        return CJT_OK;
    }
    // two passes: 2048 complex values per workgroup in the column pass (TC
    // columns of L1) and TU row pairs of L2 (at least 2048 values) in the row pass;
    // every thread holds 16 values of one transform.
    const int TC = std::max(1, 2048 / g.L1);
    const int TU = std::max(1, 1024 / g.L2);
    const int nth1 = TC * (g.L1 / 16), nth2 = 2 * TU * (g.L2 / 16);
    if (g.L2 % TC != 0 || (g.L1 / 2) % TU != 0 || nth1 > 256 || nth2 > 256 || TU * g.L2 != nth2 * kEPT)
        return fail(CJT_EUNSUPPORTED, "FFT split not supported");
    const size_t lds1 = (size_t)TC * slice_stride(g.L1) * esz;
    const size_t acc_off = ((size_t)2 * TU * slice_stride(g.L2) * esz + 255) & ~(size_t)255;
    const size_t lds2 = acc_off + sizeof(double) * (2 * kEPT + 1) * nth2;
    cjt_status st = allow_lds(k_pass1<T, S>, lds1);
    if (st == CJT_OK) st = allow_lds(k_pass2<T, K>, lds2);
    if (st != CJT_OK) return st;
    dim3 g1(g.L2 / TC, max_jobs, a.count);
    {
        ProfScope ps(a.name1, a.flops1, a.bytes1, a.stream);
        hipLaunchKernelGGL((k_pass1<T, S>), g1, dim3(nth1), lds1, a.stream, a.d_desc, g, TC);
        CJT_HIP_TRY(hipGetLastError());
    }
    dim3 g2((g.L1 / 2) / TU, 1, a.count);
    {
        ProfScope ps(a.name2, a.flops2, a.bytes2, a.stream);
        hipLaunchKernelGGL((k_pass2<T, K>), g2, dim3(nth2), lds2, a.stream, a.d_desc, g, TU, max_jobs,
                           single_job ? 1 : 0, acc_off);
        CJT_HIP_TRY(hipGetLastError());
    }
    return CJT_OK;
}

}  // namespace

cjt_status launch_rdft(const EngineArgs& a, Src src, Sink sink, bool fp32)
{
    if (src == Src::FwdAsy && sink == Sink::FwdAsy)
        return fp32 ? run<float, Src::FwdAsy, Sink::FwdAsy>(a) : run<double, Src::FwdAsy, Sink::FwdAsy>(a);
    if (src == Src::InvAsy && sink == Sink::InvAsy)
        return fp32 ? run<float, Src::InvAsy, Sink::InvAsy>(a) : run<double, Src::InvAsy, Sink::InvAsy>(a);
    if (src == Src::FwdFinal && sink == Sink::FwdFinal) return run<double, Src::FwdFinal, Sink::FwdFinal>(a);
    if (src == Src::InvInit && sink == Sink::InvInit) return run<double, Src::InvInit, Sink::InvInit>(a);
    if (src == Src::Moments && sink == Sink::Weights) return run<double, Src::Moments, Sink::Weights>(a);
    return fail(CJT_EINVAL, "unknown transform pairing");
}

// chirp-z tables: c_t = e^{i pi t^2 / L} (t < L), utw_s = e^{i pi s / L} (s <= L)
template <typename T>
__global__ void k_chirp_tables(cx<T>* chirp, cx<T>* utw, int64_t L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > L) return;
    double sn, cs;
    if (t < L) {
        const int64_t r = (t * t) % (2 * L);  // exact angle reduction
        sincospi((double)r / (double)L, &sn, &cs);
        chirp[t] = {(T)cs, (T)sn};
    }
    sincospi((double)t / (double)L, &sn, &cs);
    utw[t] = {(T)cs, (T)sn};
}

template <typename T>
__global__ void k_to_float(const cx<double>* in, cx<float>* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = {(float)in[i].re, (float)in[i].im};
}

// F(b~) in one workgroup for P <= kSingleMax
__global__ void __launch_bounds__(256) k_bl_single(FftGeom g, cx<double>* bl)
{
    extern __shared__ unsigned char smem_raw[];
    cx<double>* buf = reinterpret_cast<cx<double>*>(smem_raw);
    const int64_t P = g.P, L = g.L;
    const cx<double>* chirp = reinterpret_cast<const cx<double>*>(g.chirp);
    const cx<double>* tw = reinterpret_cast<const cx<double>*>(g.tw);
    for (int64_t t = threadIdx.x; t < P; t += blockDim.x) {
        cx<double> x = {0.0, 0.0};
        if (t < L) x = conj(chirp[t]);
        else if (t > P - L) x = conj(chirp[P - t]);
        buf[lds_pad((int)t)] = x;
    }
    __syncthreads();
    lds_fft<double>(buf, g.logP, 1, tw, 2 * P);
    for (int64_t t = threadIdx.x; t < P; t += blockDim.x) bl[t] = buf[lds_pad((int)t)];
}

// Builds chirp, utw and F(b~) for g (whose L, P, split and tw are set), in FP64
// and, if fp32, converts them.  Device memory is owned by the caller's cache.
cjt_status make_chirp_tables(FftGeom* g, bool fp32, hipStream_t st)
{
    const int64_t L = g->L, P = g->P;
    cx<double>* chirp = nullptr;
    cx<double>* utw = nullptr;
    cx<double>* bl = nullptr;
    CJT_HIP_TRY(hipMalloc(&chirp, sizeof(cx<double>) * L));
    CJT_HIP_TRY(hipMalloc(&utw, sizeof(cx<double>) * (L + 1)));
    CJT_HIP_TRY(hipMalloc(&bl, sizeof(cx<double>) * P));
    hipLaunchKernelGGL(k_chirp_tables<double>, dim3((unsigned)((L + 1 + 255) / 256)), dim3(256), 0, st, chirp, utw, L);
    CJT_HIP_TRY(hipGetLastError());
    FftGeom g64 = *g;
    g64.chirp = chirp;
    g64.utw = utw;
    const void* tw64 = nullptr;
    cjt_status s = CJT_OK;
    if (fp32) {
        // the kernel spectrum is always formed in FP64
        s = fft_twiddles_cached(P, false, st, &tw64);
        if (s != CJT_OK) return s;
        g64.tw = tw64;
    }
    if (g->single) {
        const size_t lds = lds_bytes((int)P, sizeof(cx<double>));
        s = allow_lds(k_bl_single, lds);
        if (s != CJT_OK) return s;
        hipLaunchKernelGGL(k_bl_single, dim3(1), dim3(256), lds, st, g64, bl);
        CJT_HIP_TRY(hipGetLastError());
    } else {
        cx<double>* scratch = nullptr;
        CJT_HIP_TRY(hipMalloc(&scratch, sizeof(cx<double>) * P));
        const int TC = std::max(1, 2048 / g->L1), TR = std::max(1, 2048 / g->L2);
        const int nth1 = TC * (g->L1 / 16), nth2 = TR * (g->L2 / 16);
        const size_t lds1 = (size_t)TC * slice_stride(g->L1) * 16, lds2 = (size_t)TR * slice_stride(g->L2) * 16;
        s = allow_lds(k_bs_col<double, Src::FwdAsy, 0>, lds1);
        if (s == CJT_OK) s = allow_lds(k_bs_row<double, Src::FwdAsy, 0>, lds2);
        if (s != CJT_OK) return s;
        hipLaunchKernelGGL((k_bs_col<double, Src::FwdAsy, 0>), dim3(g->L2 / TC, 1, 1), dim3(nth1), lds1, st,
                           (const ExecDesc*)nullptr, g64, TC, scratch);
        CJT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL((k_bs_row<double, Src::FwdAsy, 0>), dim3(g->L1 / TR, 1, 1), dim3(nth2), lds2, st,
                           (const ExecDesc*)nullptr, g64, TR, scratch, bl);
        CJT_HIP_TRY(hipGetLastError());
        CJT_HIP_TRY(hipStreamSynchronize(st));
        CJT_HIP_TRY(hipFree(scratch));
    }
    if (!fp32) {
        g->chirp = chirp;
        g->utw = utw;
        g->bl = bl;
    } else {
        cx<float>* c32 = nullptr;
        cx<float>* u32 = nullptr;
        cx<float>* b32 = nullptr;
        CJT_HIP_TRY(hipMalloc(&c32, sizeof(cx<float>) * L));
        CJT_HIP_TRY(hipMalloc(&u32, sizeof(cx<float>) * (L + 1)));
        CJT_HIP_TRY(hipMalloc(&b32, sizeof(cx<float>) * P));
        hipLaunchKernelGGL(k_to_float<float>, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, chirp, c32, L);
        hipLaunchKernelGGL(k_to_float<float>, dim3((unsigned)((L + 256) / 256)), dim3(256), 0, st, utw, u32, L + 1);
        hipLaunchKernelGGL(k_to_float<float>, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, bl, b32, P);
        CJT_HIP_TRY(hipGetLastError());
        CJT_HIP_TRY(hipStreamSynchronize(st));
        CJT_HIP_TRY(hipFree(chirp));
        CJT_HIP_TRY(hipFree(utw));
        CJT_HIP_TRY(hipFree(bl));
        g->chirp = c32;
        g->utw = u32;
        g->bl = b32;
    }
    CJT_HIP_TRY(hipStreamSynchronize(st));
    return CJT_OK;
}

size_t fft_job_bytes(int64_t L, bool fp32)
{
    const size_t esz = fp32 ? 8 : 16;
    if ((L & (L - 1)) == 0) return L > kSingleMax ? esz * (size_t)L : 0;
    int64_t P = 1;
    while (P < 2 * L - 1) P <<= 1;
    return P > kSingleMax ? esz * (size_t)(2 * P + L) : 0;
}

// tw[q] = exp(i pi q / L), q < 2L
template <typename T>
__global__ void k_twiddle(cx<T>* tw, int64_t L)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= 2 * L) return;
    double s, c;
    sincospi((double)q / (double)L, &s, &c);
    tw[q] = {(T)c, (T)s};
}

cjt_status make_twiddles(int64_t L, bool fp32, const void** out, hipStream_t stream)
{
    void* p = nullptr;
    const size_t bytes = (size_t)(2 * L) * (fp32 ? sizeof(cx<float>) : sizeof(cx<double>));
    CJT_HIP_TRY(hipMalloc(&p, bytes));
    const int64_t n = 2 * L;
    dim3 grid((unsigned)((n + 255) / 256));
    if (fp32) hipLaunchKernelGGL(k_twiddle<float>, grid, dim3(256), 0, stream, (cx<float>*)p, L);
    else hipLaunchKernelGGL(k_twiddle<double>, grid, dim3(256), 0, stream, (cx<double>*)p, L);
    CJT_HIP_TRY(hipGetLastError());
    *out = p;
    return CJT_OK;
}

}  // namespace cjt
