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
// terms (m) and blocks (k) of its rows and accumulates in LDS, so each output
// is written once.  Lengths that are not powers of two go through the chirp-z
// identity with the same power-of-two passes.
//
// Every kernel works on a flat list of work items (descriptor, job, tile), so
// one launch serves any mix of degrees; the geometry of each instance's
// length is read from its descriptor.
#include <algorithm>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <type_traits>

#include "cjt_internal.h"
#include "fft_lds.h"

namespace cjt {

// ------------------------------------------------------------------ sources
//
// Indices inside one transform are 32-bit (lengths are at most 2^23); a
// half-open range test lo <= n < hi is one unsigned compare.

__device__ __forceinline__ bool in_range(int n, int lo, int hi) { return (unsigned)(n - lo) < (unsigned)(hi - lo); }

// a += v as its own rounding: v passes through an empty register barrier, so
// no product inside v is fused with this add.  Sums over the jobs of an
// instance therefore round the same way whether one workgroup adds them in
// turn or a reduce adds per-job parts in the same order.
__device__ __forceinline__ void accum(double& a, double v)
{
    asm volatile("" : "+v"(v));
    a += v;
}

template <Src S>
struct Source;

template <>
struct Source<Src::FwdAsy> {
    // job = k * M + m
    static constexpr bool kMulti = true;
    // Branch-free: one pair of loads at an always valid address, masked by
    // the block's degree range, so all loads of a thread issue back to back.
    __device__ static cx<double> load(const ExecDesc& d, int job, int t)
    {
        const int k = job / d.M, m = job - k * d.M;
        const int lo = (int)d.deg_lo[k], hi = (int)d.deg_hi[k];
        const int N = (int)d.N;
        const int n0 = 2 * t, n1 = n0 + 1;
        const int c0 = min(n0, N - 1);  // pair (c0, c0 + 1) within [0, N]
        const double* Cm = d.C + (int64_t)m * (d.N + 1);
        const dpair8 c = ldg_pair(Cm + c0), x = ldg_pair(d.in + c0);
        const double v0 = n0 == c0 ? c.x * x.x : c.y * x.y;  // n0 = N reads the upper element
        const double v1 = c.y * x.y;
        return {in_range(n0, lo, hi) ? v0 : 0.0, in_range(n1, lo, hi) ? v1 : 0.0};
    }
    // (C_{n,m} c_n) at n = 2t, 2t+1 for every block at once (degrees above N
    // hold a stand-in that every block's mask clears)
    __device__ static cx<double> term(const ExecDesc& d, int m, int t)
    {
        const int N = (int)d.N;
        const int n0 = 2 * t, c0 = min(n0, N - 1);
        const double* Cm = d.C + (int64_t)m * (d.N + 1);
        const dpair8 c = ldg_pair(Cm + c0), x = ldg_pair(d.in + c0);
        return {n0 == c0 ? c.x * x.x : c.y * x.y, c.y * x.y};
    }
    // block k keeps its degrees [deg_lo, deg_hi)
    template <typename T>
    __device__ static cx<T> keep(const ExecDesc& d, int k, int t, cx<T> z)
    {
        const int lo = (int)d.deg_lo[k], hi = (int)d.deg_hi[k];
        return {in_range(2 * t, lo, hi) ? z.re : (T)0, in_range(2 * t + 1, lo, hi) ? z.im : (T)0};
    }
};

template <>
struct Source<Src::InvAsy> {
    static constexpr bool kMulti = true;
    // With a_j = u_m(theta_j) g_j and b_j = v_m(theta_j) g_j on the window (zero
    // elsewhere): r_0 = a_0, r_G = a_G, r_j = (a_j + b_j)/2 and
    // r_{2G-j} = (a_j - b_j)/2 for 0 < j < G.  The plan stores the halved sum and
    // difference of (u_m, v_m) as two planes S and D of G+1 values (both ends
    // are outside every window, where u_m = v_m = 0), so r_j = S_j g_j for
    // j <= G and r_{2G-j} = D_j g_j.
    __device__ static cx<double> load(const ExecDesc& d, int job, int t)
    {
        const int k = job / d.M;
        return pair(d, k, job - k * d.M, t);
    }
    // (r_q, r_{q+1}) of term m on block k's window for q = 2t.  Both come from
    // the adjacent points jl, jl + 1: q < G takes S at q, q+1; q >= G takes D at
    // the mirrors 2G-q, 2G-q-1 (D_G = S_G = 0 covers q = G).  Two pair loads at
    // always valid addresses, then masks; the S pair is 16-byte aligned (q even)
    // and so is the D pair (G even, jl odd, plane offset G+1).
    __device__ static cx<double> pair(const ExecDesc& d, int k, int m, int t)
    {
        const int lo = (int)d.win_lo[k], hi = (int)d.win_hi[k] + 1;
        const int G = (int)d.G;
        const double* S = reinterpret_cast<const double*>(d.uv + (int64_t)m * (G + 1));
        const int q = 2 * t;
        const bool upper = q >= G;
        const int jl = upper ? 2 * G - q - 1 : q;  // in [0, G - 1]
        const dpair8 g = ldg_pair(d.p + jl);
        const dpair8 w = ldg_pair(S + (upper ? G + 1 : 0) + jl);
        const double a0 = w.x * g.x, a1 = w.y * g.y;  // at points jl, jl + 1
        const int j0 = upper ? jl + 1 : jl, j1 = upper ? jl : jl + 1;
        const double r0 = upper ? a1 : a0, r1 = upper ? a0 : a1;
        return {in_range(j0, lo, hi) ? r0 : 0.0, in_range(j1, lo, hi) ? r1 : 0.0};
    }
    // the pair on block 0's window, which holds every other block's window
    __device__ static cx<double> term(const ExecDesc& d, int m, int t) { return pair(d, 0, m, t); }
    // block k keeps the points of its own window
    template <typename T>
    __device__ static cx<T> keep(const ExecDesc& d, int k, int t, cx<T> z)
    {
        const int lo = (int)d.win_lo[k], hi = (int)d.win_hi[k] + 1;
        const int G = (int)d.G, q = 2 * t;
        const int j0 = q <= G ? q : 2 * G - q, j1 = q + 1 <= G ? q + 1 : 2 * G - q - 1;
        return {in_range(j0, lo, hi) ? z.re : (T)0, in_range(j1, lo, hi) ? z.im : (T)0};
    }
};

template <>
struct Source<Src::FwdFinal> {
    static constexpr bool kMulti = false;
    // p = recurrence part + Hahn-block part (the latter only if the plan has blocks)
    __device__ static double pv(const ExecDesc& d, int j) { return d.nblk > 0 ? ldg(d.p + j) + ldg(d.p2 + j) : ldg(d.p + j); }
    __device__ static cx<double> load(const ExecDesc& d, int, int t)
    {
        const int N = (int)d.N, j0 = 2 * t, j1 = j0 + 1;
        const double x0 = j0 <= N ? pv(d, j0) * ((j0 == 0 || j0 == N) ? 0.5 : 1.0) : 0.0;
        const double x1 = j1 <= N ? pv(d, j1) * ((j1 == N) ? 0.5 : 1.0) : 0.0;
        return {x0, x1};
    }
};

template <>
struct Source<Src::InvInit> {
    static constexpr bool kMulti = false;
    __device__ static cx<double> load(const ExecDesc& d, int, int t)
    {
        const int N = (int)d.N, k0 = 2 * t, k1 = k0 + 1;
        return {k0 <= N ? ldg(d.in + k0) : 0.0, k1 <= N ? ldg(d.in + k1) : 0.0};
    }
};

template <>
struct Source<Src::Moments> {
    static constexpr bool kMulti = false;
    // in = mu_0..mu_G, halved at both ends
    __device__ static cx<double> load(const ExecDesc& d, int, int t)
    {
        const int G = (int)d.G, k0 = 2 * t, k1 = k0 + 1;
        const double x0 = k0 <= G ? ldg(d.in + k0) * ((k0 == 0 || k0 == G) ? 0.5 : 1.0) : 0.0;
        const double x1 = k1 <= G ? ldg(d.in + k1) * ((k1 == G) ? 0.5 : 1.0) : 0.0;
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
    __device__ static double contrib(const ExecDesc& d, int job, int i, cx<double> X)
    {
        const int k = job / d.M, m = job - k * d.M;
        if (!in_range(i, (int)d.win_lo[k], (int)d.win_hi[k] + 1)) return 0.0;
        const cx<double> uv = ldg(d.uv + (int64_t)m * (d.G + 1) + i);
        return fma(uv.re, X.re, uv.im * X.im);
    }
    // every point is written (zero outside the windows); the final DCT-I adds
    // the recurrence part
    __device__ static void finish(const ExecDesc& d, int i, double v) { stg(d.p2 + i, v); }
};

template <>
struct Target<Sink::InvAsy> {
    __device__ static double contrib(const ExecDesc& d, int job, int n, cx<double> X)
    {
        const int k = job / d.M, m = job - k * d.M;
        if (!in_range(n, (int)d.deg_lo[k], (int)d.deg_hi[k])) return 0.0;
        return ldg(d.C + (int64_t)m * (d.N + 1) + n) * (X.re + X.im);
    }
    // Every degree 0..N is written (zero outside the blocks); the recurrence
    // reduction adds its part and applies 1/A_n afterwards.
    __device__ static void finish(const ExecDesc& d, int n, double v)
    {
        if (n <= d.N) stg(d.out + n, v);
    }
};

template <>
struct Target<Sink::FwdFinal> {
    __device__ static double contrib(const ExecDesc&, int, int, cx<double> X) { return X.re; }
    __device__ static void finish(const ExecDesc& d, int k, double v)
    {
        const int N = (int)d.N;
        const double sc = (k == 0 || k == N) ? 1.0 / (double)N : 2.0 / (double)N;
        stg(d.out + k, sc * v);
    }
};

template <>
struct Target<Sink::InvInit> {
    __device__ static double contrib(const ExecDesc&, int, int, cx<double> X) { return X.re; }
    __device__ static void finish(const ExecDesc& d, int j, double v) { stg(d.p + j, ldg(d.w + j) * v); }
};

template <>
struct Target<Sink::Weights> {
    __device__ static double contrib(const ExecDesc&, int, int, cx<double> X) { return X.re; }
    // w_j = (1 - (d_j0 + d_jG)/2) / (G/2) Re X_j
    __device__ static void finish(const ExecDesc& d, int j, double v)
    {
        const int G = (int)d.G;
        const double sc = ((j == 0 || j == G) ? 0.5 : 1.0) / (0.5 * (double)G);
        stg(d.out + j, sc * v);
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

// ------------------------------------------------------------------ helpers

template <typename T>
__device__ __forceinline__ cx<T> to_t(cx<double> v) { return {(T)v.re, (T)v.im}; }

template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) { return {a.re * s, a.im * s}; }

// Geometry of an instance's length in the arithmetic precision T.
template <typename T>
__device__ __forceinline__ const FftGeom& geom_of(const ExecDesc& d);
template <>
__device__ __forceinline__ const FftGeom& geom_of<double>(const ExecDesc& d) { return d.geo; }
template <>
__device__ __forceinline__ const FftGeom& geom_of<float>(const ExecDesc& d) { return d.geob; }

// X_s and X_{L-s} of the real-input DFT from the complex FFT Z (any L; s <= L/2).
template <typename T, typename ZAt>
__device__ __forceinline__ void untangle_at(ZAt Z, int L, int s, cx<T> w, cx<double>& xa, cx<double>& xb)
{
    if (s == 0) {
        const cx<T> z = Z(0);
        xa = {(double)z.re + (double)z.im, 0.0};
        xb = {(double)z.re - (double)z.im, 0.0};
    } else if (2 * s == L) {
        const cx<T> z = Z(s);
        xa = {(double)z.re, (double)z.im};
        xb = xa;
    } else {
        untangle<T>(Z(s), Z(L - s), w, xa, xb);
    }
}

// Column twiddles.  Thread lt of column n2 holds outputs k1 = lt + u sigma
// (u = F1/16, sigma = 0..15 a permutation of its 16 register slots), which
// are multiplied by e^{2 pi i n2 k1 / F} = a b^sigma with a = e^{2 pi i n2 lt/F}
// and b = e^{2 pi i n2 u/F}: two reads of the length-F table per thread, and
// b^sigma = B^(sigma >> 2) b^(sigma & 3), B = b^4, from a few products (at
// most six roundings per twiddle).
template <typename T>
struct ColTw {
    cx<T> A[4];  // a B^h
    cx<T> p[4];  // b^l
    __device__ __forceinline__ void init(const cx<T>* __restrict__ tw, int F, int n2, int lt, int u)
    {
        const int mask = 2 * F - 1;
        const cx<T> a = ldg(tw + ((2 * n2 * lt) & mask));
        const cx<T> b = ldg(tw + ((2 * n2 * u) & mask));
        p[0] = {(T)1, (T)0};
        p[1] = b;
        p[2] = cmul(b, b);
        p[3] = cmul(p[2], b);
        const cx<T> B = cmul(p[2], p[2]), B2 = cmul(B, B);
        A[0] = a;
        A[1] = cmul(a, B);
        A[2] = cmul(a, B2);
        A[3] = cmul(A[2], B);
    }
};

// Stores the 16 outputs of fft_reg (last radix 2^LR) of column n2, times the
// column twiddles: slot s holds k1 = lt + u sigma(s).
template <int LR, typename T, typename StoreF>
__device__ __forceinline__ void col_store(cx<T> (&v)[16], const ColTw<T>& ct, int lt, int u, int lg2, int n2,
                                          StoreF store)
{
    constexpr int R = 1 << LR;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int sigma = (s >> LR) + ((s & (R - 1)) << (4 - LR));
        const int k1 = lt + u * sigma;
        store((k1 << lg2) + n2, cmul(v[s], cmul(ct.A[sigma >> 2], ct.p[sigma & 3])));
    }
}

template <typename T, typename StoreF>
__device__ __forceinline__ void col_store_any(cx<T> (&v)[16], const ColTw<T>& ct, int lt, int lg1, int lg2, int n2,
                                              StoreF store)
{
    const int u = 1 << (lg1 - 4);
    switch (fft_last_log_radix(lg1)) {
    case 4: col_store<4>(v, ct, lt, u, lg2, n2, store); break;
    case 3: col_store<3>(v, ct, lt, u, lg2, n2, store); break;
    case 2: col_store<2>(v, ct, lt, u, lg2, n2, store); break;
    default: col_store<1>(v, ct, lt, u, lg2, n2, store); break;
    }
}

// Column pass of a power-of-two FFT of length F = F1 F2 (F1 = 2^lg1 <= 2048,
// F2 = 2^lg2): TC = 2048 / F1 columns per workgroup of 128 threads; thread lt
// of column c holds n1 = lt + r F1/16.  Output k1 of column n2 is multiplied by
// e^{2 pi i n2 k1 / F}.  load(t) gives input t = n1 F2 + n2; store(k1 F2 + n2, v).
// tw: table of length F (column twiddles); tw1: table of length F1 (stages).
template <typename T, typename LoadF, typename StoreF>
__device__ __forceinline__ void col_pass(cx<T>* lds, int lg1, int lg2, const cx<T>* __restrict__ tw,
                                         const cx<T>* __restrict__ tw1, int tile, LoadF load, StoreF store)
{
    const int F1 = 1 << lg1;
    const int F = 1 << (lg1 + lg2);
    const int ltc = lg1 >= 11 ? 0 : 11 - lg1;  // TC = 2048 / F1 columns
    const int tid = threadIdx.x;
    const int c = tid & ((1 << ltc) - 1), lt = tid >> ltc;
    const int col = (tile << ltc) + c;
    const int step = F1 >> 4;
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = load(((lt + r * step) << lg2) + col);
    ColTw<T> ct;
    ct.init(tw, F, col, lt, step);
    fft_reg<T>(v, lds + c * slice_stride(F1), lg1, lt, true, tw1, 2 * F1);
    col_store_any<T>(v, ct, lt, lg1, lg2, col, store);
}

// Row pass: TR = max(1, 2048 / F2) rows k1 per workgroup (F2/16 threads each);
// load(k1 F2 + n2), store(k1 + F1 k2, X) in natural frequency order.
// tw2: table of length F2 (stages).
template <typename T, typename LoadF, typename StoreF>
__device__ __forceinline__ void row_pass(cx<T>* lds, int lg1, int lg2, const cx<T>* __restrict__ tw2, int tile,
                                         LoadF load, StoreF store)
{
    const int F2 = 1 << lg2;
    const int ltr = lg2 >= 11 ? 0 : 11 - lg2;  // TR = 2048 / F2 rows
    const int ltp = lg2 - 4;                    // threads per row: F2 / 16
    const int tid = threadIdx.x;
    const int rr = tid >> ltp, lt = tid & ((1 << ltp) - 1);
    const int k1 = (tile << ltr) + rr;
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = load((k1 << lg2) + lt + (r << ltp));
    fft_reg<T>(v, lds + rr * slice_stride(F2), lg2, lt, true, tw2, 2 * F2);
#pragma unroll
    for (int s = 0; s < 16; ++s) store(k1 + (fft_out_index(s, lt, lg2) << lg1), v[s]);
}

// ------------------------------------------------------------------ power of two, one workgroup

// One workgroup per instance; the whole length-L transform lives in LDS.
// Loops over all jobs of the instance and accumulates per thread in LDS.
template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_single(const ExecDesc* __restrict__ descs, const Item* __restrict__ items,
                                                size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[items[blockIdx.x].desc];
    const FftGeom& g = geom_of<T>(d);
    const int L = (int)g.L;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const int nel = L / 2 + 1;  // elements s = 0..L/2
    double* acc = reinterpret_cast<double*>(smem_raw + acc_off);
    for (int i = 0; i < kSlots; ++i) acc[i * nth + tid] = 0.0;
    const int njobs = Source<S>::kMulti ? d.nblk * d.M : 1;
    for (int iter = 0; iter < njobs; ++iter) {
        // terms m outer, blocks k inner: the order of the two-pass and job-parallel sums
        const int job = Source<S>::kMulti ? (iter % d.nblk) * d.M + iter / d.nblk : 0;
        for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = to_t<T>(Source<S>::load(d, job, t));
        __syncthreads();
        lds_fft<T>(buf, g.logL, 1, tw, 2 * g.L);
#pragma unroll 2
        for (int q = 0; q < kSlots / 2; ++q) {
            const int s = tid + q * nth;
            if (s >= nel) break;
            cx<double> xa, xb;
            untangle_at<T>([&](int i) { return buf[lds_pad(i)]; }, L, s, ldg(tw + s), xa, xb);
            accum(acc[(2 * q) * nth + tid], Target<K>::contrib(d, job, s, xa));
            if (2 * s != L) accum(acc[(2 * q + 1) * nth + tid], Target<K>::contrib(d, job, L - s, xb));
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

// ------------------------------------------------------------------ power of two, two passes

// Column pass, item (desc, job, column tile): writes tmp[job][k1 L2 + n2].
// Items come tile-major (all jobs of a tile together, terms m outer) and are
// spread over the XCDs in contiguous ranges, so the jobs of one tile read the
// shared inputs (g, c_n, the diagonals of a term) from the same L2.
template <typename T, Src S>
__global__ void __launch_bounds__(128) k_pass1(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Item it = items[xcd_item(blockIdx.x, gridDim.x)];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int job = it.a;
    cx<T>* out = reinterpret_cast<cx<T>*>(d.tmp) + (int64_t)job * g.L;
    col_pass<T>(
        lds, g.logL1, g.logL2, reinterpret_cast<const cx<T>*>(g.tw), reinterpret_cast<const cx<T>*>(g.tw1), it.b,
        [&](int t) { return to_t<T>(Source<S>::load(d, job, t)); }, [&](int i, cx<T> v) { stg(out + i, v); });
}

// Column pass of every Hahn block of one term, item (desc, term m, column
// tile).  The inputs of term m (forward: C_{n,m} c_n; inverse: the pair on
// block 0's window, which holds every other block's window) are gathered
// once into registers; each block k then clears what lies outside its own
// degrees (forward) or window (inverse), transforms, and writes tmp[k M + m].
// This reads the inputs once per term instead of once per (block, term).
template <typename T, Src S>
__global__ void __launch_bounds__(128) k_pass1_terms(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* lds = reinterpret_cast<cx<T>*>(smem_raw);
    const Item it = items[xcd_item(blockIdx.x, gridDim.x)];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int m = it.a;
    const int lg1 = g.logL1, lg2 = g.logL2;
    const int F1 = 1 << lg1, F = 1 << (lg1 + lg2);
    const int ltc = lg1 >= 11 ? 0 : 11 - lg1;  // TC = 2048 / F1 columns
    const int tid = threadIdx.x;
    const int c = tid & ((1 << ltc) - 1), lt = tid >> ltc;
    const int col = (it.b << ltc) + c;
    const int step = F1 >> 4;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const cx<T>* tw1 = reinterpret_cast<const cx<T>*>(g.tw1);
    cx<T> z[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = to_t<T>(Source<S>::term(d, m, ((lt + r * step) << lg2) + col));
    for (int k = 0; k < d.nblk; ++k) {
        // indices and addresses are recomputed per block: z alone stays live
        const int ltk = opaque(lt), colk = opaque(col);
        cx<T> v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = Source<S>::template keep<T>(d, k, ((ltk + r * step) << lg2) + colk, z[r]);
        fft_reg<T>(v, lds + c * slice_stride(F1), lg1, ltk, true, tw1, 2 * F1);
        // column twiddles after the transform, so they hold no registers across it
        ColTw<T> ct;
        ct.init(tw, F, colk, ltk, step);
        cx<T>* out = reinterpret_cast<cx<T>*>(d.tmp) + (int64_t)(k * d.M + m) * g.L;
        col_store_any<T>(v, ct, ltk, lg1, lg2, colk, [&](int i, cx<T> x) { stg(out + i, x); });
    }
}

// Per-job parts of the row pass (job-parallel mode): after the two-pass
// intermediates of every job, L + 1 doubles per job in iteration order.
template <typename T>
__device__ __forceinline__ double* row_parts(const ExecDesc& d, int L)
{
    return reinterpret_cast<double*>(reinterpret_cast<cx<T>*>(d.tmp) + (int64_t)d.nblk * d.M * L);
}

// Row pass, item (desc, iteration, unit tile, one_job): TU units per
// workgroup; unit u holds rows u and L1-u (unit 0 holds rows 0 and L1/2).
// Element (u, k2) pairs Z at row u, position k2 with Z at row L1-u, position
// L2-1-k2, which are Z_s and Z_{L-s} for s = u + L1 k2.  The L2-point FFTs run
// in registers; their outputs go through LDS once so each thread can fetch
// both members of its pairs.
//
// Normally a workgroup sums every job of its rows.  In job-parallel mode
// (one_job, for calls with few instances, where the row tiles alone cannot
// fill the GPU) it takes only iteration `iteration` and stores that job's
// part; k_job_row_reduce then adds the parts in iteration order, which is
// the order and association of the fused sum, so both modes give bitwise the
// same results.
template <typename T, Sink K, bool kMulti>
__global__ void __launch_bounds__(256) k_pass2(const ExecDesc* __restrict__ descs, const Item* __restrict__ items,
                                               size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int L1 = g.L1, L2 = g.L2;
    const int L = (int)g.L;
    const int TU = L2 >= 1024 ? 1 : 1024 / L2;
    const int unit0 = it.b * TU;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const int tpr = L2 >> 4;  // threads per row
    const int rs = tid / tpr, lt = tid - rs * tpr;
    const int my_unit = unit0 + (rs >> 1);
    const int my_row = (rs & 1) == 0 ? my_unit : (my_unit == 0 ? L1 / 2 : L1 - my_unit);
    constexpr int ept = kEPT;  // TU * L2 regular elements per workgroup, kEPT per thread
    const bool has_half = (unit0 == 0) && (tid == nth - 1);  // thread that also owns s = L/2
    const int sst = slice_stride(L2);

    double* acc = reinterpret_cast<double*>(smem_raw + acc_off);
    for (int i = 0; i <= 2 * ept; ++i) acc[i * nth + tid] = 0.0;

    // jobs in the order (m, k), k fastest, so that the diagonals of term m are
    // re-read from L2 for every block
    const int njobs = kMulti ? d.nblk * d.M : 1;
    const bool one_job = kMulti && it.c != 0;
    const int iter0 = one_job ? it.a : 0, iter1 = one_job ? it.a + 1 : njobs;
    for (int iter = iter0; iter < iter1; ++iter) {
        const int job = kMulti ? (iter % d.nblk) * d.M + iter / d.nblk : 0;
        // addresses are recomputed per job rather than held across the loop
        const int ltj = opaque(lt), tidj = opaque(tid);
        const cx<T>* in = reinterpret_cast<const cx<T>*>(d.tmp) + (int64_t)job * L + (int64_t)my_row * L2;
        cx<T> v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = ldg(in + ltj + r * tpr);
        cx<T>* slice = buf + rs * sst;
        fft_reg<T>(v, slice, g.logL2, ltj, true, reinterpret_cast<const cx<T>*>(g.tw2), 2 * L2);
#pragma unroll
        for (int s = 0; s < 16; ++s) slice[lds_pad(fft_out_index(s, ltj, g.logL2))] = v[s];
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < ept; ++q) {
            const int eps = tidj + q * nth;
            const int lu = eps % TU, k2 = eps / TU;
            const int unit = unit0 + lu;
            const int ra = 2 * lu, rb = 2 * lu + 1;
            cx<double> xa, xb;
            int s;
            if (unit == 0) {
                if (k2 < L2 / 2) {
                    s = L1 / 2 + L1 * k2;
                    untangle<T>(buf[rb * sst + lds_pad(k2)], buf[rb * sst + lds_pad(L2 - 1 - k2)], ldg(tw + s), xa, xb);
                } else if (k2 == L2 / 2) {
                    s = 0;
                    cx<T> z = buf[ra * sst];
                    xa = {(double)z.re + (double)z.im, 0.0};
                    xb = {(double)z.re - (double)z.im, 0.0};
                } else {
                    const int kk = k2 - L2 / 2;
                    s = L1 * kk;
                    untangle<T>(buf[ra * sst + lds_pad(kk)], buf[ra * sst + lds_pad(L2 - kk)], ldg(tw + s), xa, xb);
                }
            } else {
                s = unit + L1 * k2;
                untangle<T>(buf[ra * sst + lds_pad(k2)], buf[rb * sst + lds_pad(L2 - 1 - k2)], ldg(tw + s), xa, xb);
            }
            accum(acc[(2 * q) * nth + tidj], Target<K>::contrib(d, job, s, xa));
            accum(acc[(2 * q + 1) * nth + tidj], Target<K>::contrib(d, job, L - s, xb));
        }
        if (has_half) {
            cx<T> z = buf[lds_pad(L2 / 2)];  // row 0, position L2/2: s = L/2
            accum(acc[(2 * ept) * nth + tid], Target<K>::contrib(d, job, L / 2, cx<double>{(double)z.re, (double)z.im}));
        }
        __syncthreads();
    }
    double* part = one_job ? row_parts<T>(d, L) + (int64_t)it.a * (L + 1) : nullptr;
    auto put = [&](int s, double v) {
        if (part) stg(part + s, v);
        else Target<K>::finish(d, s, v);
    };
#pragma unroll
    for (int q = 0; q < ept; ++q) {
        const int eps = tid + q * nth;
        const int lu = eps % TU, k2 = eps / TU;
        const int unit = unit0 + lu;
        int s;
        if (unit == 0) {
            if (k2 < L2 / 2) s = L1 / 2 + L1 * k2;
            else if (k2 == L2 / 2) s = 0;
            else s = L1 * (k2 - L2 / 2);
        } else {
            s = unit + L1 * k2;
        }
        put(s, acc[(2 * q) * nth + tid]);
        put(L - s, acc[(2 * q + 1) * nth + tid]);
    }
    if (has_half) put(L / 2, acc[(2 * ept) * nth + tid]);
}

// item (desc, 0, tile of 256 outputs): the row pass's per-job parts added in
// iteration order (terms m outer, blocks k inner), then the sink
template <typename T, Sink K>
__global__ void __launch_bounds__(256) k_job_row_reduce(const ExecDesc* __restrict__ descs,
                                                        const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const int L = (int)geom_of<T>(d).L;
    const int s = it.b * blockDim.x + threadIdx.x;
    if (s > L) return;
    const double* part = row_parts<T>(d, L);
    const int njobs = d.nblk * d.M;
    double acc = 0.0;
    for (int iter = 0; iter < njobs; ++iter) accum(acc, ldg(part + (int64_t)iter * (L + 1) + s));
    Target<K>::finish(d, s, acc);
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
// Job storage (complex, 2P per job): [0, P) column-pass output; [P, 2P) the
// first transform in natural order, then Z in [P, P+L) after the second.

template <typename T>
__device__ __forceinline__ cx<T>* bs_job(const ExecDesc& d, const FftGeom& g, int job)
{
    return reinterpret_cast<cx<T>*>(d.tmp) + (int64_t)job * 2 * g.P;
}

// first transform, column pass: input a_t = source(t) c_t (zero for t >= L)
template <typename T, Src S>
__global__ void __launch_bounds__(128) k_bs_col1(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    const Item it = items[xcd_item(blockIdx.x, gridDim.x)];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int job = it.a;
    const int L = (int)g.L;
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    cx<T>* base = bs_job<T>(d, g, job);
    col_pass<T>(
        reinterpret_cast<cx<T>*>(smem_raw), g.logL1, g.logL2, reinterpret_cast<const cx<T>*>(g.tw),
        reinterpret_cast<const cx<T>*>(g.tw1), it.b,
        [&](int t) {
            return t < L ? cmul(to_t<T>(Source<S>::load(d, job, t)), ldg(chirp + t)) : cx<T>{(T)0, (T)0};
        },
        [&](int i, cx<T> v) { stg(base + i, v); });
}

// Twiddle e^{2 pi i n k / F} of slot s after fft_reg (output n = lt + u sigma(s))
// from the two-read power split of ColTw.
template <int LR, typename T>
__device__ __forceinline__ cx<T> slot_twiddle(const ColTw<T>& ct, int s)
{
    constexpr int R = 1 << LR;
    const int sigma = (s >> LR) + ((s & (R - 1)) << (4 - LR));
    return cmul(ct.A[sigma >> 2], ct.p[sigma & 3]);
}

// Row pass of the convolution, in place on rows k1 (TR rows per workgroup):
// the L2-point FFT of row k1 gives A at frequencies k1 + L1 k2; times the kernel
// spectrum (stored row-major, [k1][k2]); the inverse L2-point FFT along the same
// row (conjugate, forward FFT, conjugate) and the inverse column twiddle
// e^{-2 pi i n2 k1 / P} leave B'[k1][n2], whose inverse column FFTs give the
// convolution in natural order.  Replaces a row pass, a column pass and a row
// pass of the plain two-transform form.
template <typename T>
__global__ void __launch_bounds__(256) k_bs_rowconv(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    cx<T>* base = bs_job<T>(d, g, it.a);
    const int lg2 = g.logL2;
    const int F2 = 1 << lg2;
    const int ltr = lg2 >= 11 ? 0 : 11 - lg2;  // TR = 2048 / F2 rows
    const int ltp = lg2 - 4;                    // threads per row: F2 / 16
    const int tid = threadIdx.x;
    const int rr = tid >> ltp, lt = tid & ((1 << ltp) - 1);
    const int k1 = (it.b << ltr) + rr;
    cx<T>* slice = reinterpret_cast<cx<T>*>(smem_raw) + rr * slice_stride(F2);
    const cx<T>* tw2 = reinterpret_cast<const cx<T>*>(g.tw2);
    const cx<T>* blT = reinterpret_cast<const cx<T>*>(g.bl) + ((int64_t)k1 << lg2);
    cx<T>* row = base + ((int64_t)k1 << lg2);
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = ldg(row + lt + (r << ltp));
    fft_reg<T>(v, slice, lg2, lt, true, tw2, 2 * F2);
    // v[s] = A_{k1 + L1 k2}, k2 = fft_out_index(s): product with the kernel
    // spectrum, conjugated, redistributed for the second row FFT
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int k2 = fft_out_index(s, lt, lg2);
        slice[lds_pad(k2)] = conj(cmul(v[s], ldg(blT + k2)));
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = slice[lds_pad(lt + (r << ltp))];
#pragma unroll
    for (int r = 0; r < 16; ++r) lds_pin(v[r]);
    __syncthreads();
    fft_reg<T>(v, slice, lg2, lt, true, tw2, 2 * F2);
    // v[s] = conj(B[k1][n2]), n2 = lt + u sigma(s); store B e^{-2 pi i n2 k1 / P}
    ColTw<T> ct;
    const int u = F2 >> 4;
    ct.init(reinterpret_cast<const cx<T>*>(g.tw), (int)g.P, k1, lt, u);
    auto put = [&](auto lrc) {
        constexpr int LR = decltype(lrc)::value;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
            const int sigma = (s >> LR) + ((s & ((1 << LR) - 1)) << (4 - LR));
            stg(row + lt + u * sigma, conj(cmul(v[s], slot_twiddle<LR, T>(ct, s))));
        }
    };
    switch (fft_last_log_radix(lg2)) {
    case 4: put(std::integral_constant<int, 4>{}); break;
    case 3: put(std::integral_constant<int, 3>{}); break;
    case 2: put(std::integral_constant<int, 2>{}); break;
    default: put(std::integral_constant<int, 1>{}); break;
    }
}

// Inverse column pass of the convolution: for column n2, the inverse L1-point
// FFT over k1 of B'[k1][n2] (conjugate, forward FFT, conjugate) gives the
// convolution at n1 L2 + n2; Z_s = c_s (a * b)_s / P for s < L goes to [P, P+L).
template <typename T>
__global__ void __launch_bounds__(128) k_bs_col2inv(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    const Item it = items[xcd_item(blockIdx.x, gridDim.x)];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    cx<T>* base = bs_job<T>(d, g, it.a);
    const int P = (int)g.P, L = (int)g.L;
    const int lg1 = g.logL1, lg2 = g.logL2;
    const int F1 = 1 << lg1;
    const int ltc = lg1 >= 11 ? 0 : 11 - lg1;  // TC = 2048 / F1 columns
    const int tid = threadIdx.x;
    const int c = tid & ((1 << ltc) - 1), lt = tid >> ltc;
    const int n2 = (it.b << ltc) + c;
    const int step = F1 >> 4;
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    const T invP = (T)1 / (T)P;
    cx<T> v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = conj(ldg(base + (((lt + r * step) << lg2) + n2)));
    fft_reg<T>(v, reinterpret_cast<cx<T>*>(smem_raw) + c * slice_stride(F1), lg1, lt, true,
               reinterpret_cast<const cx<T>*>(g.tw1), 2 * F1);
#pragma unroll
    for (int s = 0; s < 16; ++s) {
        const int t = (fft_out_index(s, lt, lg1) << lg2) + n2;
        if (t < L) stg(base + P + t, cmul(ldg(chirp + t), cscale(conj(v[s]), invP)));
    }
}

// Untangling of the length-2L real DFT from Z, summed over the jobs of the
// instance (terms m outer, blocks k inner); item (desc, tile of 256 elements
// (s, L-s)).
template <typename T, Sink K, bool kMulti>
__global__ void __launch_bounds__(256) k_bs_untangle(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int L = (int)g.L;
    const int64_t P = g.P;
    const int s = it.b * blockDim.x + threadIdx.x;
    if (s > L / 2) return;
    const cx<T>* utw = reinterpret_cast<const cx<T>*>(g.utw);
    const int njobs = kMulti ? d.nblk * d.M : 1;
    double a0 = 0.0, a1 = 0.0;
    for (int iter = 0; iter < njobs; ++iter) {
        const int job = kMulti ? (iter % d.nblk) * d.M + iter / d.nblk : 0;
        const cx<T>* Z = reinterpret_cast<const cx<T>*>(d.tmp) + (int64_t)job * 2 * P + P;
        cx<double> xa, xb;
        untangle_at<T>([&](int i) { return ldg(Z + i); }, L, s, ldg(utw + s), xa, xb);
        accum(a0, Target<K>::contrib(d, job, s, xa));
        if (2 * s != L) accum(a1, Target<K>::contrib(d, job, L - s, xb));
    }
    Target<K>::finish(d, s, a0);
    if (2 * s != L) Target<K>::finish(d, L - s, a1);
}

// Whole chirp-z transform in one workgroup (P <= kSingleMax), looping over the jobs.
template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_bs_single(const ExecDesc* __restrict__ descs, const Item* __restrict__ items,
                                                   size_t acc_off)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const ExecDesc& d = descs[items[blockIdx.x].desc];
    const FftGeom& g = geom_of<T>(d);
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
    const int njobs = Source<S>::kMulti ? d.nblk * d.M : 1;
    for (int iter = 0; iter < njobs; ++iter) {
        // terms m outer, blocks k inner: the order of the two-pass and job-parallel sums
        const int job = Source<S>::kMulti ? (iter % d.nblk) * d.M + iter / d.nblk : 0;
        for (int t = tid; t < P; t += nth)
            buf[lds_pad(t)] = t < L ? cmul(to_t<T>(Source<S>::load(d, job, t)), ldg(chirp + t)) : cx<T>{(T)0, (T)0};
        __syncthreads();
        lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
        for (int t = tid; t < P; t += nth) buf[lds_pad(t)] = conj(cmul(buf[lds_pad(t)], ldg(bl + t)));
        __syncthreads();
        lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
        for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = cmul(ldg(chirp + t), cscale(conj(buf[lds_pad(t)]), invP));
        __syncthreads();
#pragma unroll 2
        for (int q = 0; q < kSlots / 2; ++q) {
            const int sx = tid + q * nth;
            if (sx >= nel) break;
            cx<double> xa, xb;
            untangle_at<T>([&](int i) { return buf[lds_pad(i)]; }, L, sx, ldg(utw + sx), xa, xb);
            accum(acc[(2 * q) * nth + tid], Target<K>::contrib(d, job, sx, xa));
            if (2 * sx != L) accum(acc[(2 * q + 1) * nth + tid], Target<K>::contrib(d, job, L - sx, xb));
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

// ------------------------------------------------------------------ job-parallel single workgroup
//
// For calls with few instances the single-workgroup kinds run one workgroup
// per (instance, job): the transform of that job, its untangling and its sink
// contributions, written to part[job][s] (doubles, s = 0..L); a second kernel
// adds the jobs in a fixed order and stores the result.

template <typename T>
__device__ __forceinline__ double* job_part(const ExecDesc& d, int job)
{
    return reinterpret_cast<double*>(d.tmp) + (int64_t)job * (d.geo.L + 1);
}

template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_single_job(const ExecDesc* __restrict__ descs, const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int job = it.a;
    const int L = (int)g.L;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = to_t<T>(Source<S>::load(d, job, t));
    __syncthreads();
    lds_fft<T>(buf, g.logL, 1, tw, 2 * g.L);
    double* part = job_part<T>(d, job);
    for (int s = tid; s <= L / 2; s += nth) {
        cx<double> xa, xb;
        untangle_at<T>([&](int i) { return buf[lds_pad(i)]; }, L, s, ldg(tw + s), xa, xb);
        stg(part + s, Target<K>::contrib(d, job, s, xa));
        if (2 * s != L) stg(part + L - s, Target<K>::contrib(d, job, L - s, xb));
    }
}

template <typename T, Src S, Sink K>
__global__ void __launch_bounds__(256) k_bs_single_job(const ExecDesc* __restrict__ descs,
                                                       const Item* __restrict__ items)
{
    extern __shared__ unsigned char smem_raw[];
    cx<T>* buf = reinterpret_cast<cx<T>*>(smem_raw);
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const FftGeom& g = geom_of<T>(d);
    const int job = it.a;
    const int L = (int)g.L, P = (int)g.P;
    const int tid = threadIdx.x, nth = blockDim.x;
    const cx<T>* tw = reinterpret_cast<const cx<T>*>(g.tw);
    const cx<T>* chirp = reinterpret_cast<const cx<T>*>(g.chirp);
    const cx<T>* bl = reinterpret_cast<const cx<T>*>(g.bl);
    const cx<T>* utw = reinterpret_cast<const cx<T>*>(g.utw);
    const T invP = (T)1 / (T)P;
    for (int t = tid; t < P; t += nth)
        buf[lds_pad(t)] = t < L ? cmul(to_t<T>(Source<S>::load(d, job, t)), ldg(chirp + t)) : cx<T>{(T)0, (T)0};
    __syncthreads();
    lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
    for (int t = tid; t < P; t += nth) buf[lds_pad(t)] = conj(cmul(buf[lds_pad(t)], ldg(bl + t)));
    __syncthreads();
    lds_fft<T>(buf, g.logP, 1, tw, 2 * g.P);
    for (int t = tid; t < L; t += nth) buf[lds_pad(t)] = cmul(ldg(chirp + t), cscale(conj(buf[lds_pad(t)]), invP));
    __syncthreads();
    double* part = job_part<T>(d, job);
    for (int s = tid; s <= L / 2; s += nth) {
        cx<double> xa, xb;
        untangle_at<T>([&](int i) { return buf[lds_pad(i)]; }, L, s, ldg(utw + s), xa, xb);
        stg(part + s, Target<K>::contrib(d, job, s, xa));
        if (2 * s != L) stg(part + L - s, Target<K>::contrib(d, job, L - s, xb));
    }
}

// item (desc, tile of 256 outputs): sum over jobs, terms m outer and blocks k inner
template <Sink K>
__global__ void __launch_bounds__(256) k_job_reduce(const ExecDesc* __restrict__ descs,
                                                    const Item* __restrict__ items)
{
    const Item it = items[blockIdx.x];
    const ExecDesc& d = descs[it.desc];
    const int L = (int)d.geo.L;
    const int s = it.b * blockDim.x + threadIdx.x;
    if (s > L) return;
    const int njobs = d.nblk * d.M;
    double acc = 0.0;
    for (int iter = 0; iter < njobs; ++iter) {
        const int job = (iter % d.nblk) * d.M + iter / d.nblk;
        accum(acc, ldg(reinterpret_cast<const double*>(d.tmp) + (int64_t)job * (L + 1) + s));
    }
    Target<K>::finish(d, s, acc);
}

// ------------------------------------------------------------------ host side

namespace {

size_t lds_bytes(int64_t n_elems, size_t esz) { return (size_t)(n_elems + (n_elems >> 4) + 1) * esz; }
size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }
int clamp_nth(int64_t F) { return (int)std::min<int64_t>(256, std::max<int64_t>(64, F / 16)); }

// Workgroups of this engine use up to ~110 KB of LDS (gfx950 has 160 KB per CU);
// the dynamic-LDS limit of a kernel is raised once per device and size, so a
// launch sequence replayed under stream capture makes no attribute calls.
std::mutex g_lds_mu;
std::map<std::pair<int, const void*>, size_t> g_lds_set;

template <typename K>
cjt_status allow_lds(K kernel, size_t bytes)
{
    int dev = 0;
    CJT_HIP_TRY(hipGetDevice(&dev));
    const void* f = reinterpret_cast<const void*>(kernel);
    std::lock_guard<std::mutex> lk(g_lds_mu);
    size_t& cur = g_lds_set[{dev, f}];
    if (bytes <= cur) return CJT_OK;
    CJT_HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    cur = bytes;
    return CJT_OK;
}

// Timing labels live as long as the library (a handful of distinct strings).
const char* intern(const std::string& x)
{
    static std::mutex mu;
    static std::set<std::string> names;
    std::lock_guard<std::mutex> lk(mu);
    return names.insert(x).first->c_str();
}

template <typename K, typename... Args>
cjt_status go(K kernel, const Launch& L, hipStream_t s, Args... args)
{
    if (L.nitems <= 0) return CJT_OK;
    if (L.lds > 48 * 1024) {
        cjt_status st = allow_lds(kernel, L.lds);
        if (st != CJT_OK) return st;
    }
    ProfScope ps(L.name, L.flops, L.bytes, s);
    hipLaunchKernelGGL(kernel, dim3((unsigned)L.nitems), dim3(L.nth), L.lds, s, args...);
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

template <typename T, Src S, Sink K>
cjt_status run(const Launch& L, const ExecDesc* dd, const Item* it, hipStream_t s)
{
    constexpr bool kMulti = Source<S>::kMulti;
    switch (L.kind) {
    case Kind::FftSingle: return go(k_single<T, S, K>, L, s, dd, it, L.acc_off);
    case Kind::FftPass1: return go(k_pass1<T, S>, L, s, dd, it);
    case Kind::FftPass1Terms:
        if constexpr (S == Src::InvAsy || S == Src::FwdAsy) return go(k_pass1_terms<T, S>, L, s, dd, it);
        return fail(CJT_EINVAL, "multi-block column pass is for the Hahn blocks");
    case Kind::FftPass2: return go(k_pass2<T, K, kMulti>, L, s, dd, it, L.acc_off);
    case Kind::JobRowReduce:
        if constexpr (kMulti) return go(k_job_row_reduce<T, K>, L, s, dd, it);
        return fail(CJT_EINVAL, "per-job row parts are for the Hahn blocks");
    case Kind::BsSingle: return go(k_bs_single<T, S, K>, L, s, dd, it, L.acc_off);
    case Kind::BsCol1: return go(k_bs_col1<T, S>, L, s, dd, it);
    case Kind::BsRowConv: return go(k_bs_rowconv<T>, L, s, dd, it);
    case Kind::BsCol2Inv: return go(k_bs_col2inv<T>, L, s, dd, it);
    case Kind::BsUntangle: return go(k_bs_untangle<T, K, kMulti>, L, s, dd, it);
    case Kind::FftJobs: return go(k_single_job<T, S, K>, L, s, dd, it);
    case Kind::BsJobs: return go(k_bs_single_job<T, S, K>, L, s, dd, it);
    case Kind::JobReduce: return go(k_job_reduce<K>, L, s, dd, it);
    default: return fail(CJT_EINVAL, "not an FFT launch");
    }
}

}  // namespace

cjt_status launch_fft(const Launch& L, const ExecDesc* dd, const Item* it, hipStream_t s)
{
    const bool f = L.fp32 != 0;
    if (L.src == Src::FwdAsy && L.sink == Sink::FwdAsy)
        return f ? run<float, Src::FwdAsy, Sink::FwdAsy>(L, dd, it, s) : run<double, Src::FwdAsy, Sink::FwdAsy>(L, dd, it, s);
    if (L.src == Src::InvAsy && L.sink == Sink::InvAsy)
        return f ? run<float, Src::InvAsy, Sink::InvAsy>(L, dd, it, s) : run<double, Src::InvAsy, Sink::InvAsy>(L, dd, it, s);
    if (f) return fail(CJT_EINVAL, "boundary transforms run in FP64");
    if (L.src == Src::FwdFinal && L.sink == Sink::FwdFinal) return run<double, Src::FwdFinal, Sink::FwdFinal>(L, dd, it, s);
    if (L.src == Src::InvInit && L.sink == Sink::InvInit) return run<double, Src::InvInit, Sink::InvInit>(L, dd, it, s);
    if (L.src == Src::Moments && L.sink == Sink::Weights) return run<double, Src::Moments, Sink::Weights>(L, dd, it, s);
    return fail(CJT_EINVAL, "unknown transform pairing");
}

// The job-parallel mode applies to single-workgroup lengths with more than
// one job; add_fft and fft_tmp_bytes decide it with this one predicate.
static bool job_mode(const FftGeom& g, int64_t jobs, bool job_parallel)
{
    return job_parallel && jobs > 1 && g.single;
}

// The row pass of a two-pass power-of-two transform takes one job per
// workgroup (and a reduce) in calls with few instances, for lengths whose
// row tiles alone (L / 2048 per instance) cannot fill the GPU; same
// predicate for add_fft and fft_tmp_bytes.
static bool row_job_mode(const FftGeom& g, int64_t jobs, bool job_parallel)
{
    return job_parallel && jobs > 1 && !g.single && !g.bluestein && g.L < ((int64_t)1 << 19);
}

// Job of iteration `it` in the order terms m outer, blocks k inner.
static int job_at(const ExecDesc& d, int it, bool multi)
{
    return multi ? (it % d.nblk) * d.M + it / d.nblk : 0;
}

// Launch classes of one engine pass: instances are bucketed by kernel and
// workgroup size; each bucket is one launch over its items.
cjt_status add_fft(Program& pr, const std::vector<int>& which, Src src, Sink sink, bool fp32, int stream,
                   const char* name_cols, const char* name_rows, const std::vector<double>& flops,
                   const std::vector<double>& bytes, bool job_parallel)
{
    const bool multi = (src == Src::FwdAsy || src == Src::InvAsy);
    const bool f32 = fp32 && multi;
    const size_t esz = f32 ? sizeof(cx<float>) : sizeof(cx<double>);
    struct Bucket {
        Kind kind;
        int nth;
        std::vector<Item> items;
        size_t lds = 0, acc = 0;
        double flops = 0, bytes = 0;
        const char* name;
    };
    std::vector<Bucket> bk;
    auto bucket = [&](Kind k, int nth, const char* nm) -> Bucket& {
        for (auto& b : bk)
            if (b.kind == k && b.nth == nth) return b;
        bk.push_back(Bucket{k, nth, {}, 0, 0, 0, 0, nm});
        return bk.back();
    };
    for (int i : which) {
        const ExecDesc& d = pr.descs[i];
        const FftGeom& g = f32 ? d.geob : d.geo;
        const int jobs = multi ? d.nblk * d.M : 1;
        if (jobs <= 0) continue;
        const double fl = flops[i], by = bytes[i];
        if (multi && job_mode(g, jobs, job_parallel)) {
            const int64_t F = g.bluestein ? g.P : g.L;
            Bucket& b = bucket(g.bluestein ? Kind::BsJobs : Kind::FftJobs, clamp_nth(F), name_cols);
            for (int j = 0; j < jobs; ++j) b.items.push_back(Item{i, j, 0, 0});
            b.lds = std::max(b.lds, lds_bytes(F, esz));
            b.flops += 0.5 * fl;
            b.bytes += 0.5 * by;
            Bucket& br = bucket(Kind::JobReduce, 256, name_rows);
            for (int64_t t = 0; t < (g.L + 1 + 255) / 256; ++t) br.items.push_back(Item{i, 0, (int32_t)t, 0});
            br.flops += 0.5 * fl;
            br.bytes += 0.5 * by;
        } else if (!g.bluestein && g.single) {
            const int nth = clamp_nth(g.L);
            if ((g.L / 2 + 1 + nth - 1) / nth > kSlots / 2) return fail(CJT_EUNSUPPORTED, "single-pass length");
            Bucket& b = bucket(Kind::FftSingle, nth, name_cols);
            b.items.push_back(Item{i, 0, 0, 0});
            b.acc = std::max(b.acc, a256(lds_bytes(g.L, esz)));
            b.flops += fl;
            b.bytes += by;
        } else if (!g.bluestein) {
            if (g.L1 > 2048 || g.L2 > 2048) return fail(CJT_EUNSUPPORTED, "FFT length too large");
            const int TC = g.L1 >= 2048 ? 1 : 2048 / g.L1;
            const int TU = g.L2 >= 1024 ? 1 : 1024 / g.L2;
            const int nth2 = 2 * TU * (g.L2 / 16);
            // one item per term (all blocks of the term in the workgroup), except
            // for forward calls with few instances, where one item per (block,
            // term) gives a single long transform K times the workgroups
            const bool terms = multi && (src == Src::InvAsy || !job_parallel);
            Bucket& b1 = bucket(terms ? Kind::FftPass1Terms : Kind::FftPass1, 128, name_cols);
            for (int t = 0; t < g.L2 / TC; ++t) {
                if (terms) {
                    for (int m = 0; m < d.M; ++m) b1.items.push_back(Item{i, m, t, 0});
                } else {
                    for (int it = 0; it < jobs; ++it) b1.items.push_back(Item{i, job_at(d, it, multi), t, 0});
                }
            }
            b1.lds = std::max(b1.lds, (size_t)TC * slice_stride(g.L1) * esz);
            b1.flops += 0.5 * fl;
            b1.bytes += 0.5 * by;
            Bucket& b2 = bucket(Kind::FftPass2, nth2, name_rows);
            const bool one_job = multi && row_job_mode(g, jobs, job_parallel);
            for (int q = 0; q < (one_job ? jobs : 1); ++q)
                for (int t = 0; t < (g.L1 / 2) / TU; ++t) b2.items.push_back(Item{i, q, t, one_job ? 1 : 0});
            b2.acc = std::max(b2.acc, a256((size_t)2 * TU * slice_stride(g.L2) * esz));
            b2.flops += 0.5 * fl;
            b2.bytes += 0.5 * by;
            if (one_job) {
                Bucket& br = bucket(Kind::JobRowReduce, 256, name_rows);
                for (int64_t t = 0; t < (g.L + 1 + 255) / 256; ++t) br.items.push_back(Item{i, 0, (int32_t)t, 0});
            }
        } else if (g.single) {
            const int nth = clamp_nth(g.P);
            if ((g.L / 2 + 1 + nth - 1) / nth > kSlots / 2) return fail(CJT_EUNSUPPORTED, "chirp-z length");
            Bucket& b = bucket(Kind::BsSingle, nth, name_cols);
            b.items.push_back(Item{i, 0, 0, 0});
            b.acc = std::max(b.acc, a256(lds_bytes(g.P, esz)));
            b.flops += fl;
            b.bytes += by;
        } else {
            if (g.L1 > 2048 || g.L2 > 4096) return fail(CJT_EUNSUPPORTED, "chirp-z length too large");
            const int TC = g.L1 >= 2048 ? 1 : 2048 / g.L1;
            const int TR = g.L2 >= 2048 ? 1 : 2048 / g.L2;
            const int nthr = TR * (g.L2 / 16);
            const Kind ks[3] = {Kind::BsCol1, Kind::BsRowConv, Kind::BsCol2Inv};
            for (int q = 0; q < 3; ++q) {
                const bool col = q != 1;
                Bucket& b = bucket(ks[q], col ? 128 : nthr, name_cols);
                const int tiles = col ? g.L2 / TC : g.L1 / TR;
                if (col) {  // tile-major, as the power-of-two column pass
                    for (int t = 0; t < tiles; ++t)
                        for (int it = 0; it < jobs; ++it) b.items.push_back(Item{i, job_at(d, it, multi), t, 0});
                } else {
                    for (int j = 0; j < jobs; ++j)
                        for (int t = 0; t < tiles; ++t) b.items.push_back(Item{i, j, t, 0});
                }
                b.lds = std::max(b.lds, col ? (size_t)TC * slice_stride(g.L1) * esz : (size_t)TR * slice_stride(g.L2) * esz);
                b.flops += fl / 6.0;
                b.bytes += by / 6.0;
            }
            Bucket& bu = bucket(Kind::BsUntangle, 256, name_rows);
            for (int64_t t = 0; t < (g.L / 2 + 1 + 255) / 256; ++t) bu.items.push_back(Item{i, 0, (int32_t)t, 0});
            bu.flops += 0.5 * fl;
            bu.bytes += 0.5 * by;
        }
    }
    // timing labels: the caller's column / row names, with the chirp-z and
    // single-workgroup kinds told apart
    auto label = [&](Kind k, const char* nm) -> const char* {
        if (!nm) return nullptr;
        const char* sfx = "";
        switch (k) {
        case Kind::FftSingle: sfx = "_single"; break;
        case Kind::BsSingle: sfx = "_bs_single"; break;
        case Kind::BsCol1:
        case Kind::BsCol2Inv: sfx = "_bs_cols"; break;
        case Kind::BsRowConv: sfx = "_bs_rows"; break;
        case Kind::BsUntangle: sfx = "_bs_untangle"; break;
        case Kind::FftJobs: sfx = "_jobs"; break;
        case Kind::BsJobs: sfx = "_bs_jobs"; break;
        case Kind::JobReduce: sfx = "_job_reduce"; break;
        default: break;
        }
        return intern(std::string(nm) + sfx);
    };
    // launch order: single-workgroup kinds, then the two-pass chains in dependency order
    const Kind order[] = {Kind::FftSingle, Kind::BsSingle, Kind::FftJobs, Kind::BsJobs,  Kind::JobReduce,
                          Kind::FftPass1,  Kind::FftPass1Terms, Kind::FftPass2, Kind::JobRowReduce, Kind::BsCol1,
                          Kind::BsRowConv, Kind::BsCol2Inv, Kind::BsUntangle};
    for (Kind k : order) {
        for (auto& b : bk) {
            if (b.kind != k || b.items.empty()) continue;
            Launch L;
            L.kind = k;
            L.stream = stream;
            L.src = src;
            L.sink = sink;
            L.fp32 = f32 ? 1 : 0;
            L.nth = b.nth;
            L.item_off = (int64_t)pr.items.size();
            L.nitems = (int64_t)b.items.size();
            if (k == Kind::FftSingle || k == Kind::BsSingle) {
                L.acc_off = b.acc;
                L.lds = b.acc + sizeof(double) * kSlots * b.nth;
            } else if (k == Kind::FftPass2) {
                L.acc_off = b.acc;
                L.lds = b.acc + sizeof(double) * (2 * kEPT + 1) * b.nth;
            } else {
                L.lds = b.lds;
            }
            L.name = label(k, b.name);
            L.flops = b.flops;
            L.bytes = b.bytes;
            pr.items.insert(pr.items.end(), b.items.begin(), b.items.end());
            pr.launches.push_back(L);
        }
    }
    return CJT_OK;
}

// ------------------------------------------------------------------ tables

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

// chirp-z tables: c_t = e^{i pi t^2 / L} (t < L), utw_s = e^{i pi s / L} (s <= L);
// the angle t^2 / L is reduced modulo 2 in exact integer arithmetic.
__global__ void k_chirp_tables(cx<double>* chirp, cx<double>* utw, int64_t L)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > L) return;
    double sn, cs;
    if (t < L) {
        const int64_t r = (t * t) % (2 * L);
        sincospi((double)r / (double)L, &sn, &cs);
        chirp[t] = {cs, sn};
    }
    sincospi((double)t / (double)L, &sn, &cs);
    utw[t] = {cs, sn};
}

__global__ void k_to_float(const cx<double>* in, cx<float>* out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = {(float)in[i].re, (float)in[i].im};
}

// b~_t = conj(c_|k|) wrapped cyclically: t < L, or t > P - L (k = P - t)
__device__ __forceinline__ cx<double> bl_input(const cx<double>* chirp, int64_t L, int64_t P, int64_t t)
{
    if (t < L) return conj(chirp[t]);
    if (t > P - L) return conj(chirp[P - t]);
    return {0.0, 0.0};
}

// F(b~) in one workgroup for P <= kSingleMax
__global__ void __launch_bounds__(256) k_bl_single(FftGeom g, cx<double>* bl)
{
    extern __shared__ unsigned char smem_raw[];
    cx<double>* buf = reinterpret_cast<cx<double>*>(smem_raw);
    const int64_t P = g.P, L = g.L;
    const cx<double>* chirp = reinterpret_cast<const cx<double>*>(g.chirp);
    for (int64_t t = threadIdx.x; t < P; t += blockDim.x) buf[lds_pad((int)t)] = bl_input(chirp, L, P, t);
    __syncthreads();
    lds_fft<double>(buf, g.logP, 1, reinterpret_cast<const cx<double>*>(g.tw), 2 * P);
    for (int64_t t = threadIdx.x; t < P; t += blockDim.x) bl[t] = buf[lds_pad((int)t)];
}

__global__ void __launch_bounds__(128) k_bl_col(FftGeom g, cx<double>* scratch)
{
    extern __shared__ unsigned char smem_raw[];
    const cx<double>* chirp = reinterpret_cast<const cx<double>*>(g.chirp);
    const int64_t P = g.P, L = g.L;
    col_pass<double>(
        reinterpret_cast<cx<double>*>(smem_raw), g.logL1, g.logL2, reinterpret_cast<const cx<double>*>(g.tw),
        reinterpret_cast<const cx<double>*>(g.tw1), blockIdx.x, [&](int64_t t) { return bl_input(chirp, L, P, t); }, [&](int64_t i, cx<double> v) { scratch[i] = v; });
}

// F(b~) stored row-major for the convolution row pass: frequency k1 + L1 k2 at
// [k1][k2] = k1 L2 + k2.
__global__ void __launch_bounds__(256) k_bl_row(FftGeom g, const cx<double>* scratch, cx<double>* bl)
{
    extern __shared__ unsigned char smem_raw[];
    const int64_t m1 = ((int64_t)1 << g.logL1) - 1;
    row_pass<double>(
        reinterpret_cast<cx<double>*>(smem_raw), g.logL1, g.logL2, reinterpret_cast<const cx<double>*>(g.tw2),
        blockIdx.x, [&](int64_t i) { return scratch[i]; },
        [&](int64_t i, cx<double> v) { bl[((i & m1) << g.logL2) + (i >> g.logL1)] = v; });
}

namespace {
size_t a256b(size_t x) { return (x + 255) & ~(size_t)255; }
}  // namespace

size_t chirp_table_bytes(const FftGeom& g, bool fp32)
{
    const size_t e = fp32 ? sizeof(cx<float>) : sizeof(cx<double>);
    return a256b(e * (size_t)g.L) + a256b(e * (size_t)(g.L + 1)) + a256b(e * (size_t)g.P);
}

size_t chirp_scratch_bytes(const FftGeom& g, bool fp32)
{
    size_t s = g.single ? 0 : a256b(sizeof(cx<double>) * (size_t)g.P);  // two-pass intermediate
    if (fp32) s += chirp_table_bytes(g, false);                        // FP64 tables before conversion
    return s;
}

// Builds chirp, utw and F(b~) for g (whose L, P, split and tw are set) into
// mem (chirp_table_bytes), always in FP64 first and converted for fp32; the
// construction uses scratch (chirp_scratch_bytes).  Asynchronous on st: the
// tables are ready once st reaches this point.
cjt_status make_chirp_tables(FftGeom* g, bool fp32, hipStream_t st, char* mem, char* scratch)
{
    const int64_t L = g->L, P = g->P;
    const size_t two_pass = g->single ? 0 : a256b(sizeof(cx<double>) * (size_t)P);
    char* t64 = fp32 ? scratch + two_pass : mem;
    cx<double>* chirp = (cx<double>*)t64;
    cx<double>* utw = (cx<double>*)(t64 + a256b(sizeof(cx<double>) * (size_t)L));
    cx<double>* bl = (cx<double>*)(t64 + a256b(sizeof(cx<double>) * (size_t)L) +
                                   a256b(sizeof(cx<double>) * (size_t)(L + 1)));
    hipLaunchKernelGGL(k_chirp_tables, dim3((unsigned)((L + 1 + 255) / 256)), dim3(256), 0, st, chirp, utw, L);
    CJT_HIP_TRY(hipGetLastError());
    FftGeom g64 = *g;
    g64.chirp = chirp;
    g64.utw = utw;
    cjt_status s = CJT_OK;
    if (fp32) {  // the kernel spectrum is always formed in FP64
        const void* tw64 = nullptr;
        s = fft_twiddles_cached(P, false, st, &tw64);
        if (s != CJT_OK) return s;
        g64.tw = tw64;
        if (!g->single) {
            if ((s = fft_twiddles_cached(g->L1, false, st, &g64.tw1)) != CJT_OK) return s;
            if ((s = fft_twiddles_cached(g->L2, false, st, &g64.tw2)) != CJT_OK) return s;
        }
    }
    if (g->single) {
        const size_t lds = lds_bytes(P, sizeof(cx<double>));
        s = allow_lds(k_bl_single, lds);
        if (s != CJT_OK) return s;
        hipLaunchKernelGGL(k_bl_single, dim3(1), dim3(256), lds, st, g64, bl);
        CJT_HIP_TRY(hipGetLastError());
    } else {
        cx<double>* tmp = (cx<double>*)scratch;
        const int TC = g->L1 >= 2048 ? 1 : 2048 / g->L1, TR = g->L2 >= 2048 ? 1 : 2048 / g->L2;
        const size_t lds1 = (size_t)TC * slice_stride(g->L1) * sizeof(cx<double>);
        const size_t lds2 = (size_t)TR * slice_stride(g->L2) * sizeof(cx<double>);
        s = allow_lds(k_bl_col, lds1);
        if (s == CJT_OK) s = allow_lds(k_bl_row, lds2);
        if (s != CJT_OK) return s;
        hipLaunchKernelGGL(k_bl_col, dim3(g->L2 / TC), dim3(128), lds1, st, g64, tmp);
        CJT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_bl_row, dim3(g->L1 / TR), dim3(TR * (g->L2 / 16)), lds2, st, g64, tmp, bl);
        CJT_HIP_TRY(hipGetLastError());
    }
    if (!fp32) {
        g->chirp = chirp;
        g->utw = utw;
        g->bl = bl;
    } else {
        cx<float>* c32 = (cx<float>*)mem;
        cx<float>* u32 = (cx<float>*)(mem + a256b(sizeof(cx<float>) * (size_t)L));
        cx<float>* b32 = (cx<float>*)(mem + a256b(sizeof(cx<float>) * (size_t)L) +
                                      a256b(sizeof(cx<float>) * (size_t)(L + 1)));
        hipLaunchKernelGGL(k_to_float, dim3((unsigned)((L + 255) / 256)), dim3(256), 0, st, chirp, c32, L);
        hipLaunchKernelGGL(k_to_float, dim3((unsigned)((L + 256) / 256)), dim3(256), 0, st, utw, u32, L + 1);
        hipLaunchKernelGGL(k_to_float, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, bl, b32, P);
        CJT_HIP_TRY(hipGetLastError());
        g->chirp = c32;
        g->utw = u32;
        g->bl = b32;
    }
    return CJT_OK;
}

size_t fft_tmp_bytes(const FftGeom& g, int64_t jobs, bool fp32, bool job_parallel)
{
    if (jobs <= 0) return 0;
    if (job_mode(g, jobs, job_parallel)) return sizeof(double) * (size_t)jobs * (size_t)(g.L + 1);
    const size_t parts = row_job_mode(g, jobs, job_parallel) ? sizeof(double) * (size_t)jobs * (size_t)(g.L + 1) : 0;
    return (size_t)jobs * fft_job_bytes(g.L, fp32) + parts;
}

size_t fft_job_bytes(int64_t L, bool fp32)
{
    const size_t esz = fp32 ? 8 : 16;
    if ((L & (L - 1)) == 0) return L > kSingleMax ? esz * (size_t)L : 0;
    int64_t P = 1;
    while (P < 2 * L - 1) P <<= 1;
    return P > kSingleMax ? esz * (size_t)(2 * P) : 0;
}

}  // namespace cjt
