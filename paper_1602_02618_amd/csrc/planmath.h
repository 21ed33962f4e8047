// FP64 special functions of the plan (host and device).
//
// Gamma ratios are never formed as differences of log-Gamma values (that loses
// about n*eps, Sec. 4.1); instead the Stirling-series forms of the paper are
// used: eq. Cnmabasy for the Hahn coefficients C_{n,m} and eq. Anabasy for the
// orthonormality constants A_n, with (1+x)^y evaluated as exp(y log1p(x)) and
// the series S_eps(z) truncated by Table 1.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "stirling_coeffs.h"

namespace cjt {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kEps = 2.220446049250313080847263336181640625e-16;  // 2^-52, Sec. 2.2 and Table 1

// S_eps(z) for z >= 9: Stirling's series with the number of terms of Table 1.
__host__ __device__ inline double stirling_S(double z)
{
    int nt = kStirlingTerms[CJT_STIRLING_TABLE_ROWS - 1];
    for (int r = 0; r < CJT_STIRLING_TABLE_ROWS; ++r) {
        if (z >= kStirlingZ[r]) { nt = kStirlingTerms[r]; break; }
    }
    double zi = 1.0 / z;
    double s = 0.0;
    for (int k = nt - 1; k >= 0; --k) s = fma(s, zi, kStirlingA[k]);
    return s;
}

// (1 + x)^y = exp(y log1p(x)).
__host__ __device__ inline double pow1p(double x, double y) { return exp(y * log1p(x)); }

// C_{n,m}^{a,b} (eq. Cnmab) by its Stirling form eq. Cnmabasy; valid for n + min(a,b) >= 8.
__host__ __device__ inline double hahn_C_asy(double n, int m, double a, double b)
{
    double t = 2.0 * n + a + b + m + 2.0;
    double r = exp((double)m) / (ldexp(1.0, 2 * m) * sqrt(kPi));
    r *= pow1p((a - b - m) / t, n + a + 0.5);
    r *= pow1p((b - a - m) / t, n + b + 0.5);
    r /= pow(n, m + 0.5) * pow1p((a + b + m + 2.0) / (2.0 * n), m + 0.5);
    r *= stirling_S(n + a + 1.0) * stirling_S(n + b + 1.0) / stirling_S(t);
    return r;
}

// C_{n,0} from Gamma directly (small n only, where tgamma is exact enough).
__host__ __device__ inline double hahn_C0_small(double n, double a, double b)
{
    return exp2(2.0 * n + a + b + 1.0) * tgamma(n + a + 1.0) * tgamma(n + b + 1.0) /
           (kPi * tgamma(2.0 * n + a + b + 2.0));
}

// C_{n,m}: Stirling form where valid, else Gamma at m = 0 followed by the
// m-step of eq. Cnmabrec, C_{n,m} = C_{n,m-1} / (2 (2n + a + b + m + 1)).
__host__ __device__ inline double hahn_C(double n, int m, double a, double b)
{
    if (n + fmin(a, b) >= 8.0) return hahn_C_asy(n, m, a, b);
    double c = hahn_C0_small(n, a, b);
    for (int q = 1; q <= m; ++q) c /= 2.0 * (2.0 * n + a + b + q + 1.0);
    return c;
}

// log C_{n,m}, for the partition test 2 C_{j,M} g_M(theta) < eps.
__host__ __device__ inline double hahn_logC(double n, int m, double a, double b)
{
    if (n + fmin(a, b) >= 8.0) {
        double t = 2.0 * n + a + b + m + 2.0;
        double l = (double)m - 2.0 * m * log(2.0) - 0.5 * log(kPi);
        l += (n + a + 0.5) * log1p((a - b - m) / t) + (n + b + 0.5) * log1p((b - a - m) / t);
        l -= (m + 0.5) * (log(n) + log1p((a + b + m + 2.0) / (2.0 * n)));
        l += log(stirling_S(n + a + 1.0)) + log(stirling_S(n + b + 1.0)) - log(stirling_S(t));
        return l;
    }
    return log(hahn_C(n, m, a, b));
}

// Orthonormality constant A_n (eq. Anab) by eq. Anabasy where n + min(a,b,a+b,0) >= 8,
// else by the Gamma closed form (n = 0 uses (a+b+1) Gamma(a+b+1) = Gamma(a+b+2)).
__host__ __device__ inline double jacobi_norm(double n, double a, double b)
{
    if (n + fmin(fmin(a, b), fmin(a + b, 0.0)) >= 8.0) {
        double z3 = n + a + b + 1.0, z4 = n + 1.0;
        double r = exp2(a + b + 1.0) / (2.0 * n + a + b + 1.0);
        r *= pow1p(-b / z3, 0.5 * n + a + 0.25);
        r *= pow1p(-a / z3, 0.5 * n + b + 0.25);
        r *= pow1p(a / z4, 0.5 * n + 0.25);
        r *= pow1p(b / z4, 0.5 * n + 0.25);
        r *= stirling_S(n + a + 1.0) * stirling_S(n + b + 1.0) / (stirling_S(z3) * stirling_S(z4));
        return r;
    }
    if (n == 0.0) return exp2(a + b + 1.0) * tgamma(a + 1.0) * tgamma(b + 1.0) / tgamma(a + b + 2.0);
    return exp2(a + b + 1.0) * tgamma(n + a + 1.0) * tgamma(n + b + 1.0) /
           ((2.0 * n + a + b + 1.0) * tgamma(n + a + b + 1.0) * tgamma(n + 1.0));
}

// Pochhammer products of the Hahn expansion (Sec. 2.1):
//   a_l = (1/2+a)_l (1/2-a)_l / l!,  b_l = (1/2+b)_l (1/2-b)_l / l!.
__host__ __device__ inline void hahn_pochhammer(int M, double a, double b, double* ca, double* cb)
{
    ca[0] = 1.0;
    cb[0] = 1.0;
    for (int l = 1; l <= M; ++l) {
        ca[l] = ca[l - 1] * (0.5 + a + l - 1) * (0.5 - a + l - 1) / l;
        cb[l] = cb[l - 1] * (0.5 + b + l - 1) * (0.5 - b + l - 1) / l;
    }
}

}  // namespace cjt
