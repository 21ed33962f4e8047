"""Seeded synthetic inputs for the Chebyshev--Jacobi transform.

This module only draws random numbers; it holds none of the transform's
arithmetic, so both the HIP path and the CPU oracle can be fed from it.

Every draw uses numpy's PCG64 generator (`numpy.random.default_rng(seed)`).
Per instance the draw order is: N, then alpha, then beta, then the coefficient
vector.  The paper measures on synthetic coefficients only (random Jacobi
parameters in (-1/2, 1/2) and algebraically decaying random coefficients,
Sec. 5, captions of Figs. 3 and 4); the workloads below follow that recipe.
"""
from dataclasses import dataclass
from typing import List

import numpy as np


def decaying_coeffs(rng, N, r):
    """c_n = z_n * (n+1)^(-r), z_n ~ N(0, 1), n = 0..N."""
    z = rng.standard_normal(N + 1)
    return z * (np.arange(N + 1, dtype=np.float64) + 1.0) ** (-float(r))


def log_uniform_int(rng, lo, hi):
    """floor(exp(U(ln lo, ln hi))), clipped to [lo, hi]."""
    v = int(np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
    return min(max(v, lo), hi)


@dataclass
class Instance:
    N: int
    alpha: float
    beta: float
    coeffs: np.ndarray


def single(N, alpha, beta, seed, r=1.0):
    """One transform with fixed (N, alpha, beta)."""
    rng = np.random.default_rng(seed)
    return Instance(N, float(alpha), float(beta), decaying_coeffs(rng, N, r))


def batch_uniform_params(count, N, seed, r=1.0, lo=-0.5, hi=0.5):
    """`count` transforms of one degree N with (alpha, beta) ~ U(lo, hi)^2 each."""
    rng = np.random.default_rng(seed)
    out: List[Instance] = []
    for _ in range(count):
        a = float(rng.uniform(lo, hi))
        b = float(rng.uniform(lo, hi))
        out.append(Instance(N, a, b, decaying_coeffs(rng, N, r)))
    return out


def batch_log_uniform_N(count, nlo, nhi, seed, r=1.0, lo=-0.5, hi=0.5):
    """`count` transforms with N log-uniform in [nlo, nhi] and (alpha, beta) ~ U(lo, hi)^2."""
    rng = np.random.default_rng(seed)
    out: List[Instance] = []
    for _ in range(count):
        N = log_uniform_int(rng, nlo, nhi)
        a = float(rng.uniform(lo, hi))
        b = float(rng.uniform(lo, hi))
        out.append(Instance(N, a, b, decaying_coeffs(rng, N, r)))
    return out


# The workloads the tests and the benchmark use, by name.
def small_single(seed=0):
    """N = 1024, alpha = 0.1, beta = -0.3, c_n = z_n / (n+1)."""
    return single(1024, 0.1, -0.3, seed, r=1.0)


def large_single(seed=0):
    """N = 2^20, alpha = -0.45, beta = 0.3, c_n = z_n / (n+1)^1.5."""
    return single(1 << 20, -0.45, 0.3, seed, r=1.5)


def batch_65536(seed=0, count=256):
    """256 transforms at N = 65536, (alpha, beta) ~ U(-1/2, 1/2)^2, c_n = z_n / (n+1)."""
    return batch_uniform_params(count, 65536, seed, r=1.0)


def batch_uneven(seed=0, count=4096):
    """4096 transforms, N log-uniform in [64, 16384], (alpha, beta) ~ U(-1/2, 1/2)^2."""
    return batch_log_uniform_N(count, 64, 16384, seed, r=1.0)


def serving_requests(count, seed, nlo=128, nhi=1 << 18, key_pool=0, lo=-0.5, hi=0.5):
    """Serving stream: per request the direction (forward with probability 1/2),
    N log-uniform in [nlo, nhi] and (alpha, beta) ~ U(lo, hi)^2.  With
    key_pool > 0 the (N, alpha, beta) keys are drawn once into a pool of that
    size and each request picks one uniformly.  Returns numpy arrays
    (forward: bool, N: int64, alpha, beta)."""
    rng = np.random.default_rng(seed)
    if key_pool > 0:
        keys = [(log_uniform_int(rng, nlo, nhi), float(rng.uniform(lo, hi)), float(rng.uniform(lo, hi)))
                for _ in range(key_pool)]
    fwd = np.empty(count, dtype=bool)
    N = np.empty(count, dtype=np.int64)
    a = np.empty(count)
    b = np.empty(count)
    for i in range(count):
        fwd[i] = rng.random() < 0.5
        if key_pool > 0:
            N[i], a[i], b[i] = keys[int(rng.integers(0, key_pool))]
        else:
            N[i] = log_uniform_int(rng, nlo, nhi)
            a[i] = rng.uniform(lo, hi)
            b[i] = rng.uniform(lo, hi)
    return fwd, N, a, b


def poisson_arrivals(count, rate_per_s, seed):
    """Arrival times in microseconds of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1e6 / float(rate_per_s), count))
