"""Pins for the oracle's Jacobi-to-Jacobi transform (the forward transform
followed by the inverse at other parameters, as the paper's conclusions
describe).

The independent route is the connection-coefficient lemma of Sec. 1.2 (eq.
Pnabcdconnection): P_n^(g,d) = sum_k c_{n,k}^(a,b,g,d) P_k^(a,b), evaluated in
exact rational arithmetic for dyadic parameters, so no rounding enters the
reference.  The lemma's transcription is itself checked by exact evaluation of
both sides with the textbook three-term recurrence at rational points.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

# dyadic parameters inside (-1/2, 1/2]: exact in binary, so the oracle sees the
# same values as the exact reference
A, B, G, D = Fr(1, 8), Fr(-3, 8), Fr(1, 4), Fr(7, 16)


def poch(x, k):
    r = Fr(1)
    for i in range(k):
        r *= x + i
    return r


def fact(n):
    return poch(Fr(1), n)


def connection(n, k, a, b, g, d):
    """c_{n,k}^(a,b,g,d) of eq. Pnabcdconnection, with
    Gamma(k+a+b+1) / Gamma(2k+a+b+2) = 1 / (k+a+b+1)_{k+1} and the
    terminating 3F2 at 1 summed term by term."""
    pre = poch(n + g + d + 1, k) * poch(k + g + 1, n - k) * (2 * k + a + b + 1) / (fact(n - k) * poch(k + a + b + 1, k + 1))
    s = Fr(0)
    for j in range(n - k + 1):
        s += (poch(k - n, j) * poch(n + k + g + d + 1, j) * poch(k + a + 1, j)
              / (poch(k + g + 1, j) * poch(2 * k + a + b + 2, j) * fact(j)))
    return pre * s


def jacobi_exact(nmax, a, b, x):
    """P_0..P_nmax at x by the standard three-term recurrence (exact)."""
    p = [Fr(1), ((a + b + 2) * x + (a - b)) / 2]
    for n in range(1, nmax):
        s = 2 * n + a + b
        num = (s + 1) * ((s + 2) * s * x + a * a - b * b) * p[n] - 2 * (n + a) * (n + b) * (s + 2) * p[n - 1]
        p.append(num / (2 * (n + 1) * (n + a + b + 1) * s))
    return p[: nmax + 1]


def convert_exact(coef, a, b, g, d):
    """Coefficients in P^(g,d) of sum_n coef[n] P_n^(a,b): each P_n^(a,b) is
    expanded by the lemma with the roles of the two parameter pairs swapped."""
    N = len(coef) - 1
    out = [Fr(0)] * (N + 1)
    for n in range(N + 1):
        for k in range(n + 1):
            out[k] += coef[n] * connection(n, k, g, d, a, b)
    return out


def test_connection_lemma_transcription():
    """sum_k c_{n,k} P_k^(a,b)(x) = P_n^(g,d)(x) exactly at rational x."""
    for x in (Fr(-1), Fr(-2, 3), Fr(1, 5), Fr(7, 9), Fr(1)):
        pa = jacobi_exact(7, A, B, x)
        pg = jacobi_exact(7, G, D, x)
        for n in range(8):
            assert sum(connection(n, k, A, B, G, D) * pa[k] for k in range(n + 1)) == pg[n]


def test_connection_lemma_catches_a_swap():
    """Swapping the parameter pairs gives a different expansion (the test
    above would notice the wrong direction)."""
    x = Fr(1, 5)
    pa, pg = jacobi_exact(4, A, B, x), jacobi_exact(4, G, D, x)
    assert sum(connection(4, k, G, D, A, B) * pa[k] for k in range(5)) != pg[4]


@pytest.mark.parametrize("quad", [False, True])
def test_j2j_matches_connection_coefficients(oracle_mod, quad):
    """The composition equals the exact connection-coefficient conversion."""
    rng = np.random.default_rng(7)
    N = 12
    c = rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0)
    ref = np.array([float(v) for v in convert_exact([Fr(float(v)) for v in c], A, B, G, D)])
    got = oracle_mod.jacobi_to_jacobi(c, float(A), float(B), float(G), float(D), quad=quad)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14


def test_j2j_identity_and_transitivity(oracle_mod):
    """(a, b) -> (a, b) is the identity; (a, b) -> (g, d) -> (e, f) equals
    (a, b) -> (e, f)."""
    rng = np.random.default_rng(8)
    N = 300
    c = rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0)
    a, b, g, d, e, f = 0.1, -0.3, 0.5, 0.25, -0.45, 0.3
    same = oracle_mod.jacobi_to_jacobi(c, a, b, a, b)
    assert np.linalg.norm(same - c) / np.linalg.norm(c) < 1e-14
    two = oracle_mod.jacobi_to_jacobi(oracle_mod.jacobi_to_jacobi(c, a, b, g, d), g, d, e, f)
    one = oracle_mod.jacobi_to_jacobi(c, a, b, e, f)
    assert np.linalg.norm(two - one) / np.linalg.norm(one) < 1e-14
