"""Pins for the oracle's parameter shifts (Sec. 1.2: integer increments and
decrements of the Jacobi parameters) and its inverse transform outside
(-1/2, 1/2]^2.

The shifted inverse (base inverse, then the shift relation in mpmath) is tied
to the definition itself, P c = T c_cheb at the N+1 Chebyshev--Lobatto points,
solved directly at 50 digits; the shift relation to the value identity
sum c_n P_n^(a,b)(x) = sum d_n P_n^(a0,b0)(x) evaluated with mpmath's Jacobi
functions; the forward transform at shifted parameters (its definition holds
for any a, b > -1) to mpmath's Jacobi functions."""
import mpmath as mp
import numpy as np
import pytest

PARAMS = [(1.3, -0.8), (-0.7, 2.4), (0.5, -0.5), (2.5, 1.1), (-0.9, -0.95)]


@pytest.mark.parametrize("ab", PARAMS)
def test_shift_preserves_values(oracle_mod, ab):
    a, b = ab
    N = 25
    rng = np.random.default_rng(3)
    c = rng.standard_normal(N + 1)
    d = oracle_mod.shift_coefficients(c, a, b, to_base=True)
    a0, b0 = a - np.ceil(a - 0.5), b - np.ceil(b - 0.5)
    assert -0.5 < a0 <= 0.5 and -0.5 < b0 <= 0.5
    with mp.workdps(30):
        for x in (-0.97, -0.3, 0.2, 0.88):
            lhs = mp.fsum(mp.mpf(c[n]) * mp.jacobi(n, a, b, x) for n in range(N + 1))
            rhs = mp.fsum(mp.mpf(d[n]) * mp.jacobi(n, a0, b0, x) for n in range(N + 1))
            assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    back = oracle_mod.shift_coefficients(d, a, b, to_base=False)
    assert np.allclose(back, c, rtol=1e-13, atol=1e-14)


def _definition_inverse(cheb, a, b):
    """Solve P c = T cheb at the Chebyshev--Lobatto points at 50 digits."""
    N = len(cheb) - 1
    with mp.workdps(50):
        xs = [mp.cos(mp.pi * j / N) for j in range(N + 1)]
        P = mp.matrix(N + 1, N + 1)
        rhs = mp.matrix(N + 1, 1)
        for j, x in enumerate(xs):
            for n in range(N + 1):
                P[j, n] = mp.jacobi(n, a, b, x)
            rhs[j] = mp.fsum(mp.mpf(cheb[k]) * mp.chebyt(k, x) for k in range(N + 1))
        sol = mp.lu_solve(P, rhs)
        return np.array([float(sol[n]) for n in range(N + 1)])


@pytest.mark.parametrize("ab", PARAMS)
def test_shifted_inverse_matches_definition(oracle_mod, ab):
    a, b = ab
    N = 24
    rng = np.random.default_rng(4)
    cheb = rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0)
    got = oracle_mod.inverse_shifted(cheb, a, b)
    ref = _definition_inverse(cheb, a, b)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-14


@pytest.mark.parametrize("ab", PARAMS)
def test_forward_outside_square_matches_mpmath(oracle_mod, ab):
    """Point values of the forward definition at shifted parameters."""
    a, b = ab
    N = 30
    rng = np.random.default_rng(5)
    c = rng.standard_normal(N + 1)
    pv = oracle_mod.point_values(c, a, b)
    with mp.workdps(30):
        for j in (0, 3, 11, 15, 27, 30):
            x = mp.cos(mp.pi * j / N)
            ref = mp.fsum(mp.mpf(c[n]) * mp.jacobi(n, a, b, x) for n in range(N + 1))
            assert abs(pv[j] - float(ref)) <= 1e-13 * max(1.0, abs(float(ref)))
