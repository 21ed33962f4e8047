"""ctypes wrapper and build step for the plain CPU oracle (test infrastructure only).

Every function here forwards to `cjt_oracle.c`; see that file's header for what
is computed and which passage of the paper each step follows.  `quad=True`
selects the binary128 build of the same source (unmodified recurrence at every
point, roughly 50x slower), used to check the long double build.
"""
import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cjt_oracle.c")
_LIBS = {False: os.path.join(_HERE, "libcjt_oracle.so"), True: os.path.join(_HERE, "libcjt_oracle_q.so")}
_lock = threading.Lock()
_libs = {}


def _build_one(quad):
    out = _LIBS[quad]
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]
    if quad:
        cmd += ["-DORACLE_QUAD"]
    cmd += [_SRC, "-o", out + ".tmp"]
    cmd += ["-lquadmath", "-lm"] if quad else ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build(force=True):
    """Compile the oracle with gcc (round-to-nearest, no contraction, no
    fast-math): the long double library and its binary128 cross-check build."""
    for quad in (False, True):
        lib = _LIBS[quad]
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
            _build_one(quad)
    return _LIBS[False]


def _load(quad=False):
    with _lock:
        if quad in _libs:
            return _libs[quad]
        path = _LIBS[quad]
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            _build_one(quad)
        lib = ctypes.CDLL(path)
        i64, dbl, pd, pl = ctypes.c_int64, ctypes.c_double, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        ci = ctypes.c_int
        lib.oracle_forward.argtypes = [i64, dbl, dbl, pd, pd, ci]
        lib.oracle_inverse.argtypes = [i64, dbl, dbl, pd, pd, ci]
        lib.oracle_point_values.argtypes = [i64, dbl, dbl, pd, pd, ci]
        lib.oracle_point_values_rows.argtypes = [i64, dbl, dbl, pd, i64, pl, pd, ci]
        lib.oracle_jacobi_column.argtypes = [i64, dbl, dbl, i64, i64, pd]
        lib.oracle_moments.argtypes = [i64, dbl, dbl, pd]
        lib.oracle_cc_weights.argtypes = [i64, dbl, dbl, pd, ci]
        lib.oracle_norm_consts.argtypes = [i64, dbl, dbl, pd]
        for f in ("oracle_forward", "oracle_inverse", "oracle_point_values", "oracle_point_values_rows",
                  "oracle_jacobi_column", "oracle_moments", "oracle_cc_weights", "oracle_norm_consts",
                  "oracle_version"):
            getattr(lib, f).restype = ctypes.c_int
        _libs[quad] = lib
        return lib


def default_threads():
    try:
        return max(1, min(len(os.sched_getaffinity(0)), 64))
    except AttributeError:
        return max(1, os.cpu_count() or 1)


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(st, what):
    if st != 0:
        raise RuntimeError(f"oracle {what} failed with status {st}")


def forward(c, alpha, beta, threads=None, quad=False):
    """Chebyshev coefficients T_N^{-1} P_N c of the Jacobi series c (length N+1)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    N = c.size - 1
    out = np.empty(N + 1)
    _check(_load(quad).oracle_forward(N, float(alpha), float(beta), _dp(c), _dp(out), threads or default_threads()), "forward")
    return out


def inverse(cheb, alpha, beta, threads=None, quad=False):
    """Jacobi coefficients P_N^{-1} T_N c of the Chebyshev series c (length N+1)."""
    cheb = np.ascontiguousarray(cheb, dtype=np.float64)
    N = cheb.size - 1
    out = np.empty(N + 1)
    _check(_load(quad).oracle_inverse(N, float(alpha), float(beta), _dp(cheb), _dp(out), threads or default_threads()), "inverse")
    return out


def jacobi_to_jacobi(c, alpha, beta, gamma, delta, threads=None, quad=False):
    """Coefficients in P_n^(gamma,delta) of the Jacobi series c in P_n^(alpha,beta)
    (length N+1): the forward transform at (alpha, beta) followed by the inverse
    at (gamma, delta), the composition named in the paper's conclusions.  The
    Chebyshev coefficients in between are rounded to FP64, as they are on the
    GPU path."""
    return inverse(forward(c, alpha, beta, threads, quad), gamma, delta, threads, quad)


def _split(x):
    """Integer shift s and base x - s in (-1/2, 1/2]."""
    import math
    s = math.ceil(x - 0.5)
    return s, x - s


def shift_coefficients(c, alpha, beta, to_base, dps=40):
    """Coefficients c of a Jacobi series moved between P^(alpha,beta) and the
    base family P^(alpha0,beta0), (alpha0, beta0) in (-1/2, 1/2]^2, one unit of
    parameter at a time by the relation between neighbouring parameters of
    Sec. 1.2 (for beta) and its image under x -> -x (for alpha), in mpmath at
    `dps` digits.  With A_n = (n+a+b+1)/(2n+a+b+1), A_0 = 1, and
    B_n = (n+a)/(2n+a+b+1) (beta) or -(n+b)/(2n+a+b+1) (alpha), coefficients
    d in P^(a,b) and e in the family raised by one satisfy
    e_n = A_n d_n + B_{n+1} d_{n+1}; lowering solves this from the top degree
    down.  to_base: the caller's family to the base (beta first, then alpha);
    otherwise the reverse."""
    import mpmath as mp
    with mp.workdps(dps):
        v = [mp.mpf(float(x)) for x in c]
        N = len(v) - 1
        p, a0 = _split(float(alpha))
        q, b0 = _split(float(beta))
        a0, b0 = mp.mpf(a0), mp.mpf(b0)

        def AB(n, a, b, on_a):
            if n == 0:
                return mp.mpf(1), mp.mpf(0)
            den = 2 * n + a + b + 1
            return (n + a + b + 1) / den, (-(n + b) if on_a else (n + a)) / den

        def up(a, b, on_a):
            for n in range(N + 1):
                A = AB(n, a, b, on_a)[0]
                B1 = AB(n + 1, a, b, on_a)[1]
                v[n] = A * v[n] + (B1 * v[n + 1] if n < N else 0)

        def down(a, b, on_a):
            nxt = mp.mpf(0)
            for n in range(N, -1, -1):
                A = AB(n, a, b, on_a)[0]
                B1 = AB(n + 1, a, b, on_a)[1]
                nxt = (v[n] - B1 * nxt) / A
                v[n] = nxt

        a1 = a0 + p
        if to_base:
            for j in range(q, 0, -1):
                down(a1, b0 + j - 1, False)
            for j in range(q, 0):
                up(a1, b0 + j, False)
            for i in range(p, 0, -1):
                down(a0 + i - 1, b0, True)
            for i in range(p, 0):
                up(a0 + i, b0, True)
        else:
            for i in range(0, p):
                up(a0 + i, b0, True)
            for i in range(0, p, -1):
                down(a0 + i - 1, b0, True)
            for j in range(0, q):
                up(a1, b0 + j, False)
            for j in range(0, q, -1):
                down(a1, b0 + j - 1, False)
        return np.array([float(x) for x in v])


def inverse_shifted(cheb, alpha, beta, threads=None, quad=False):
    """Inverse transform for any alpha, beta > -1: the inverse at the base
    parameters (alpha0, beta0) in (-1/2, 1/2]^2, where its moment recurrence
    is stable (Sec. 3.1), then the coefficients moved to (alpha, beta) by
    shift_coefficients.  (The forward transform needs no such route: its
    definition, evaluation by the three-term recurrence, holds for any
    alpha, beta > -1.)"""
    _, a0 = _split(float(alpha))
    _, b0 = _split(float(beta))
    return shift_coefficients(inverse(cheb, a0, b0, threads, quad), alpha, beta, to_base=False)


def point_values(c, alpha, beta, threads=None, quad=False):
    """p_j = sum_n c_n P_n(cos(pi j/N)), j = 0..N."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    N = c.size - 1
    out = np.empty(N + 1)
    _check(_load(quad).oracle_point_values(N, float(alpha), float(beta), _dp(c), _dp(out), threads or default_threads()), "point_values")
    return out


def point_values_rows(c, alpha, beta, rows, threads=None, quad=False):
    """p_j for the listed rows j only (O(N) per row)."""
    c = np.ascontiguousarray(c, dtype=np.float64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    N = c.size - 1
    out = np.empty(rows.size)
    _check(_load(quad).oracle_point_values_rows(N, float(alpha), float(beta), _dp(c), rows.size,
                                            rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out),
                                            threads or default_threads()), "point_values_rows")
    return out


def jacobi_column(nmax, alpha, beta, j, d, quad=False):
    """P_n(cos(pi j/d)) for n = 0..nmax."""
    out = np.empty(nmax + 1)
    _check(_load(quad).oracle_jacobi_column(nmax, float(alpha), float(beta), j, d, _dp(out)), "jacobi_column")
    return out


def moments(nmax, alpha, beta, quad=False):
    """Modified Chebyshev moments of the Jacobi weight, n = 0..nmax."""
    out = np.empty(nmax + 1)
    _check(_load(quad).oracle_moments(nmax, float(alpha), float(beta), _dp(out)), "moments")
    return out


def cc_weights(L, alpha, beta, threads=None, quad=False):
    """Clenshaw--Curtis weights of the Jacobi weight at cos(pi j/L), j = 0..L."""
    out = np.empty(L + 1)
    _check(_load(quad).oracle_cc_weights(L, float(alpha), float(beta), _dp(out), threads or default_threads()), "cc_weights")
    return out


def norm_consts(nmax, alpha, beta, quad=False):
    """Orthonormality constants A_n = int P_n^2 w, n = 0..nmax."""
    out = np.empty(nmax + 1)
    _check(_load(quad).oracle_norm_consts(nmax, float(alpha), float(beta), _dp(out)), "norm_consts")
    return out


def version():
    return int(_load(False).oracle_version())
