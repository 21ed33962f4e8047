// LDS-resident Stockham FFTs for gfx950 (wave64), positive exponent:
//   X_k = sum_n x_n exp(+2 pi i n k / F),  F = 2^p.
//
// A transform is split into radix-16 stages (plus one radix-8/4/2 stage when
// p is not a multiple of 4).  Every thread holds 16 complex values per stage
// in registers: one radix-16 butterfly, or 16/R radix-R butterflies.  Each stage
// reads its inputs from LDS, waits at a barrier, and writes its outputs in
// Stockham order, so the result comes out in natural order without a
// bit-reversal pass.  LDS indices are padded by one element every 16 so the
// stride-16 writes of the first stage do not serialise on one bank.
//
// Twiddles come from a table tw[q] = exp(i pi q / L), q < 2L, of the transform
// length L that this F-point transform is part of (F divides L); they are
// computed once per length from the exact rational angle, so no angle is ever
// formed by accumulation.  All lengths are powers of two up to 2^24, so
// indices and strides are 32-bit and divisions are shifts.
#pragma once

#include "cjt_internal.h"

namespace cjt {

// Keeps LDS reads on their side of the barrier that follows them.  Some
// compiler passes treat s_barrier as touching no memory and may sink a load
// whose only use lies past the barrier below it, where it races with the
// other threads' writes of the next phase.  This empty statement has side
// effects and consumes the loaded registers, so every load issued before it
// completes before it, and it stays above the barrier.  Call it once after
// all loads of a phase have been issued (they still overlap in flight).
template <typename T>
__device__ __forceinline__ void lds_pin(cx<T>& a)
{
    asm volatile("" : "+v"(a.re), "+v"(a.im));
}

// A per-thread index the compiler cannot see through.  Taken at the top of
// a loop body, it keeps the addresses derived from the index (loads, LDS
// exchanges, stores: dozens of 64-bit values in an unrolled transform) from
// being hoisted out of the loop and held in registers across all of its
// iterations, which costs waves per SIMD.
__device__ __forceinline__ int opaque(int x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ int lds_pad(int i) { return i + (i >> 4); }

// Distance between the LDS slices of consecutive transforms of length F: the
// padded length plus one element, so that threads of one wave working on
// different slices do not land on the same bank.
__host__ __device__ __forceinline__ int slice_stride(int F) { return F + (F >> 4) + 1; }

template <typename T>
__device__ __forceinline__ cx<T> cadd(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> csub(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b)
{
    return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul_i(cx<T> a) { return {-a.im, a.re}; }      // i * a
template <typename T>
__device__ __forceinline__ cx<T> cmul_mi(cx<T> a) { return {a.im, -a.re}; }     // -i * a
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.re, -a.im}; }

// In-register DFTs, positive exponent.
template <typename T>
__device__ __forceinline__ void dft2(cx<T>* v)
{
    cx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3)
{
    cx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = csub(v1, v3);
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, cmul_i(t3));
    v3 = csub(t1, cmul_i(t3));
}

template <typename T>
__device__ __forceinline__ void dft4(cx<T>* v) { dft4(v[0], v[1], v[2], v[3]); }

template <typename T>
__device__ __forceinline__ void dft8(cx<T>* v)
{
    const T h = (T)0.70710678118654752440084436210484903928;
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    // w8^k o_k, w8 = e^{i pi/4}
    cx<T> w1 = {h * (o1.re - o1.im), h * (o1.re + o1.im)};
    cx<T> w2 = cmul_i(o2);
    cx<T> w3 = {-h * (o3.re + o3.im), h * (o3.re - o3.im)};
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

template <typename T>
__device__ __forceinline__ void dft16(cx<T>* v)
{
    const T c1 = (T)0.92387953251128675612818318939678828682;  // cos(pi/8)
    const T s1 = (T)0.38268343236508977172845998403039886676;  // sin(pi/8)
    const T h = (T)0.70710678118654752440084436210484903928;
    // n = q + 4p: DFT over p for each q
#pragma unroll
    for (int q = 0; q < 4; ++q) dft4(v[q], v[q + 4], v[q + 8], v[q + 12]);
    // now v[q + 4 k1] = A_q[k1]; twiddle by w16^{q k1}
    // q = 1: k1 = 1,2,3 -> w^1, w^2, w^3
    v[5] = cmul(v[5], cx<T>{c1, s1});
    v[9] = cmul(v[9], cx<T>{h, h});
    v[13] = cmul(v[13], cx<T>{s1, c1});
    // q = 2: w^2, w^4, w^6
    v[6] = cmul(v[6], cx<T>{h, h});
    v[10] = cmul_i(v[10]);
    v[14] = cmul(v[14], cx<T>{-h, h});
    // q = 3: w^3, w^6, w^9
    v[7] = cmul(v[7], cx<T>{s1, c1});
    v[11] = cmul(v[11], cx<T>{-h, h});
    v[15] = cmul(v[15], cx<T>{-c1, -s1});
    // DFT over q for each k1: X[k1 + 4 k2]
    cx<T> o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cx<T> a0 = v[4 * k1 + 0], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
        dft4(a0, a1, a2, a3);
        o[k1] = a0;
        o[k1 + 4] = a1;
        o[k1 + 8] = a2;
        o[k1 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = o[i];
}

template <typename T, int R>
__device__ __forceinline__ void dft(cx<T>* v)
{
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// Multiplies v[r] (r = 1..R-1) by the stage twiddles w^{r k}, w^k = tw[k twmul].
// Radix 8 and 16 form them from two table reads, w^k and w^{4k}, as
// (w^{4k})^(r/4) (w^k)^(r mod 4); lower radices read each one.
template <typename T, int R>
__device__ __forceinline__ void twiddle_stage(cx<T>* v, const cx<T>* __restrict__ tw, int k, int twmul)
{
    if constexpr (R <= 4) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], ldg(tw + (r * k) * twmul));
    } else {
        const cx<T> b1 = ldg(tw + k * twmul);
        const cx<T> b4 = ldg(tw + (4 * k) * twmul);
        const cx<T> b2 = cmul(b1, b1), b3 = cmul(b2, b1);
        const cx<T> p[4] = {cx<T>{(T)1, (T)0}, b1, b2, b3};
        cx<T> a[R / 4];
        a[0] = cx<T>{(T)1, (T)0};
        a[1] = b4;
        if constexpr (R == 16) {
            a[2] = cmul(b4, b4);
            a[3] = cmul(a[2], b4);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) {
            if ((r & 3) == 0) v[r] = cmul(v[r], a[r >> 2]);
            else if (r < 4) v[r] = cmul(v[r], p[r]);
            else v[r] = cmul(v[r], cmul(a[r >> 2], p[r & 3]));
        }
    }
}

// One Stockham stage of radix R for an F-point transform at buf[base .. base+F)
// (padded indices).  `lt` is the thread's index among the F/16 threads that
// serve this transform (or 0 when F < 16), BPT = butterflies per thread.
// twmul = 2L / (Ns R) maps the stage twiddle exp(2 pi i r k / (Ns R)) into tw.
template <typename T, int R, int BPT>
__device__ __forceinline__ void fft_stage(cx<T>* buf, int F, int Ns, int lt, int base, bool active,
                                          const cx<T>* __restrict__ tw, int twmul)
{
    cx<T> v[BPT][R];
    const int FR = F / R;
    const int stride = FR / BPT;  // threads per transform
    if (active) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            int j = lt + q * stride;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[lds_pad(base + j + r * FR)];
        }
#pragma unroll
        for (int q = 0; q < BPT; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) lds_pin(v[q][r]);
    }
    __syncthreads();
    if (active) {
#pragma unroll
        for (int q = 0; q < BPT; ++q) {
            int j = lt + q * stride;
            int k = j & (Ns - 1);
            if (Ns > 1) twiddle_stage<T, R>(v[q], tw, k, twmul);
            dft<T, R>(v[q]);
            int idxD = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[lds_pad(base + idxD + r * Ns)] = v[q][r];
        }
    }
    __syncthreads();
}

// nfft transforms of size F = 2^logF stored back to back from buf[0] (padded
// indices), using threads [0, nfft * max(F/16, 1)) of the workgroup.  All
// threads of the workgroup must call this.  L2x = 2L of the parent length.
template <typename T>
__device__ __forceinline__ void lds_fft(cx<T>* buf, int logF, int nfft, const cx<T>* __restrict__ tw,
                                        int L2x)
{
    const int F = 1 << logF;
    if (logF == 0) {
        __syncthreads();
        return;
    }
    const int tpf = F >= 16 ? F / 16 : 1;
    const int tid = threadIdx.x;
    const int b = tid / tpf;
    const int lt = tid - b * tpf;
    const bool active = b < nfft;
    const int base = b * F;
    int Ns = 1;
    int rem = logF;
    while (rem > 0) {
        const int lr = rem >= 4 ? 4 : rem;
        const int twmul = L2x >> (__builtin_ctz(Ns) + lr);
        if (lr == 4) {
            fft_stage<T, 16, 1>(buf, F, Ns, lt, base, active, tw, twmul);
        } else if (F >= 16) {
            if (lr == 3) fft_stage<T, 8, 2>(buf, F, Ns, lt, base, active, tw, twmul);
            else if (lr == 2) fft_stage<T, 4, 4>(buf, F, Ns, lt, base, active, tw, twmul);
            else fft_stage<T, 2, 8>(buf, F, Ns, lt, base, active, tw, twmul);
        } else {
            if (lr == 3) fft_stage<T, 8, 1>(buf, F, Ns, lt, base, active, tw, twmul);
            else if (lr == 2) fft_stage<T, 4, 1>(buf, F, Ns, lt, base, active, tw, twmul);
            else fft_stage<T, 2, 1>(buf, F, Ns, lt, base, active, tw, twmul);
        }
        Ns <<= lr;
        rem -= lr;
    }
}

}  // namespace cjt

namespace cjt {

// ---------------------------------------------------------------------------
// Register-resident variant for F >= 16: the caller loads the first stage's
// inputs straight into registers and takes the last stage's outputs from
// registers, so only the exchanges between stages go through LDS.
//
// Thread `lt` (of F/16 per transform) holds on entry v[r] = x[lt + r F/16],
// r = 0..15.  On exit v[s] holds X[fft_out_index(s, lt, logF)].
// buf is this transform's LDS slice (F elements, padded indices).

__device__ __forceinline__ int fft_last_log_radix(int logF)
{
    const int rem = logF & 3;
    return rem == 0 ? 4 : rem;
}

// Output position of register slot s (0..15) after fft_reg.
__device__ __forceinline__ int fft_out_index(int s, int lt, int logF)
{
    const int F = 1 << logF;
    const int lr = fft_last_log_radix(logF);
    const int R = 1 << lr;
    const int q = s >> lr, r = s & (R - 1);  // butterfly q of the thread, output r
    return lt + q * (F >> 4) + r * (F >> lr);
}

template <typename T, int R, int BPT>
__device__ __forceinline__ void fft_reg_last(cx<T> (&v)[16], const cx<T>* buf, int F, int Ns, int lt,
                                             const cx<T>* __restrict__ tw, int twmul)
{
    const int FR = F / R;
    const int stride = FR / BPT;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
        const int j = lt + q * stride;
        const int k = j & (Ns - 1);
        cx<T> w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) w[r] = buf[lds_pad(j + r * FR)];
#pragma unroll
        for (int r = 0; r < R; ++r) lds_pin(w[r]);
        twiddle_stage<T, R>(w, tw, k, twmul);
        dft<T, R>(w);
#pragma unroll
        for (int r = 0; r < R; ++r) v[q * R + r] = w[r];
    }
}

// All threads of the workgroup must call this (it contains barriers); `active`
// marks threads that own a transform.
template <typename T>
__device__ __forceinline__ void fft_reg(cx<T> (&v)[16], cx<T>* buf, int logF, int lt, bool active,
                                        const cx<T>* __restrict__ tw, int L2x)
{
    const int F = 1 << logF;
    const int nst = (logF + 3) >> 2;  // stages: radix 16 ..., last one radix 2^(logF - 4(nst-1))
    if (active) dft16(v);
    if (nst == 1) return;
    // first stage output (Ns = 1): positions 16 lt + r
    if (active) {
#pragma unroll
        for (int r = 0; r < 16; ++r) buf[lds_pad(16 * lt + r)] = v[r];
    }
    __syncthreads();
    int Ns = 16;
    for (int st = 1; st + 1 < nst; ++st) {
        // middle radix-16 stages through LDS
        fft_stage<T, 16, 1>(buf, F, Ns, lt, 0, active, tw, L2x >> (__builtin_ctz(Ns) + 4));
        Ns <<= 4;
    }
    const int lr = logF - 4 * (nst - 1);
    const int twmul = L2x >> (__builtin_ctz(Ns) + lr);
    if (active) {
        if (lr == 4) fft_reg_last<T, 16, 1>(v, buf, F, Ns, lt, tw, twmul);
        else if (lr == 3) fft_reg_last<T, 8, 2>(v, buf, F, Ns, lt, tw, twmul);
        else if (lr == 2) fft_reg_last<T, 4, 4>(v, buf, F, Ns, lt, tw, twmul);
        else fft_reg_last<T, 2, 8>(v, buf, F, Ns, lt, tw, twmul);
    }
    __syncthreads();
}

}  // namespace cjt
