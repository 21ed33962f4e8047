// Integer shifts of the Jacobi parameters (Sec. 1.2).
//
// The transform core covers (alpha, beta) in (-1/2, 1/2].  An expansion in
// P^(a,b) with a or b outside that square is carried to the core's
// parameters (a0, b0) = (a - p, b - q), p and q integers, one unit at a time
// by the relation between neighbouring parameters that the paper prints,
//     (2n+a+b+1) P_n^(a,b) = (n+a+b+1) P_n^(a,b+1) + (n+a) P_{n-1}^(a,b+1),
// and its image under x -> -x (symmetry of Sec. 1.2), which moves a:
//     (2n+a+b+1) P_n^(a,b) = (n+a+b+1) P_n^(a+1,b) - (n+b) P_{n-1}^(a+1,b).
// With A_n = (n+a+b+1)/(2n+a+b+1) (A_0 = 1) and B_n the second ratio, the
// coefficients d in the lower family and e in the raised one satisfy
//     e_n = A_n d_n + B_{n+1} d_{n+1},   n = 0..N (d_{N+1} = 0),
// so raising is a two-term product and lowering the backward recurrence
//     d_n = (e_n - B_{n+1} d_{n+1}) / A_n,
// an affine recurrence solved here as a scan over 256 segments: each thread
// composes the affine map of its segment, one thread chains the maps from
// the top, and each thread replays its segment from the value entering it.
// Both run in place on one instance per workgroup, O(N) per unit shift.
#include <cmath>

#include "cjt_internal.h"
#include "plan.h"

namespace cjt {

namespace {

constexpr int kShiftThreads = 256;

struct Rel {
    double a, b;  // parameters of the lower family
    bool on_a;    // relation moving a (else b)
    __device__ double A(int64_t n) const
    {
        if (n == 0) return 1.0;
        const double dn = (double)n;
        return (dn + a + b + 1.0) / (2.0 * dn + a + b + 1.0);
    }
    __device__ double B(int64_t n) const
    {
        if (n == 0) return 0.0;
        const double dn = (double)n;
        return on_a ? -(dn + b) / (2.0 * dn + a + b + 1.0) : (dn + a) / (2.0 * dn + a + b + 1.0);
    }
};

// Coefficients in the lower family -> raised family, in place.
__device__ void raise(double* v, int64_t N, const Rel& r)
{
    for (int64_t base = 0; base <= N; base += kShiftThreads) {
        const int64_t n = base + threadIdx.x;
        const double dn = n <= N ? v[n] : 0.0;
        const double dn1 = n + 1 <= N ? v[n + 1] : 0.0;
        __syncthreads();
        if (n <= N) v[n] = fma(r.A(n), dn, r.B(n + 1) * dn1);
        __syncthreads();
    }
}

// Coefficients in the raised family -> lower family, in place.
__device__ void lower(double* v, int64_t N, const Rel& r)
{
    __shared__ double U[kShiftThreads], V[kShiftThreads], Y[kShiftThreads];
    const int t = threadIdx.x;
    const int64_t S = (N + 1 + kShiftThreads - 1) / kShiftThreads;
    const int64_t lo = min(N + 1, (int64_t)t * S), hi = min(N + 1, lo + S);
    // map of the segment: d_lo = u + w * y, y = d_hi entering from above
    double u = 0.0, w = 1.0;
    for (int64_t n = hi - 1; n >= lo; --n) {
        const double iA = 1.0 / r.A(n);
        const double c = -r.B(n + 1) * iA;
        u = fma(c, u, v[n] * iA);
        w *= c;
    }
    U[t] = u;
    V[t] = w;
    __syncthreads();
    if (t == 0) {
        double y = 0.0;  // d_{N+1}
        for (int s = kShiftThreads - 1; s >= 0; --s) {
            Y[s] = y;
            y = fma(V[s], y, U[s]);
        }
    }
    __syncthreads();
    double y = Y[t];
    for (int64_t n = hi - 1; n >= lo; --n) {
        y = (v[n] - r.B(n + 1) * y) / r.A(n);
        v[n] = y;
    }
    __syncthreads();
}

// One instance: v (N+1 coefficients) moved between P^(a0+p, b0+q) and
// P^(a0, b0).  to_base: the caller's family -> the core's (b first at
// a = a0 + p, then a at b = b0); otherwise the reverse steps in reverse order.
__global__ void __launch_bounds__(kShiftThreads) k_shift(double* v, int64_t N, double a0, double b0, int p, int q,
                                                         int to_base)
{
    const double a1 = a0 + (double)p;
    if (to_base) {
        for (int j = q; j > 0; --j) lower(v, N, Rel{a1, b0 + (double)(j - 1), false});
        for (int j = q; j < 0; ++j) raise(v, N, Rel{a1, b0 + (double)j, false});
        for (int i = p; i > 0; --i) lower(v, N, Rel{a0 + (double)(i - 1), b0, true});
        for (int i = p; i < 0; ++i) raise(v, N, Rel{a0 + (double)i, b0, true});
    } else {
        for (int i = 0; i < p; ++i) raise(v, N, Rel{a0 + (double)i, b0, true});
        for (int i = 0; i > p; --i) lower(v, N, Rel{a0 + (double)(i - 1), b0, true});
        for (int j = 0; j < q; ++j) raise(v, N, Rel{a1, b0 + (double)j, false});
        for (int j = 0; j > q; --j) lower(v, N, Rel{a1, b0 + (double)(j - 1), false});
    }
}

}  // namespace

void shift_split(double x, int* shift, double* base)
{
    const int s = (int)std::ceil(x - 0.5);
    *shift = s;
    *base = x - (double)s;
}

cjt_status apply_shift(const Plan& P, double* v, bool to_base, hipStream_t st)
{
    if (P.sh_a == 0 && P.sh_b == 0) return CJT_OK;
    hipLaunchKernelGGL(k_shift, dim3(1), dim3(kShiftThreads), 0, st, v, P.N, P.alpha, P.beta, P.sh_a, P.sh_b,
                       to_base ? 1 : 0);
    CJT_HIP_TRY(hipGetLastError());
    return CJT_OK;
}

}  // namespace cjt
