"""Jacobi-to-Jacobi transform through the C-ABI (cjt_jacobi_to_jacobi and its
batched form) against the oracle's composition, plus its identities and error
paths.

Tolerance: the composition runs the forward and the inverse transform, each
held to 1e-13 log2(N) in the relative 2-norm, and the inverse's condition on
the Chebyshev side is that of the round trip, so the bound used is twice the
single-transform tolerance."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def tol(N):
    return 2e-13 * max(math.log2(N), 1.0)


def rel2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_02618_amd import cjt
    cjt.load()
    return cjt


def coeffs(N, seed, r=1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0) ** r


@pytest.mark.parametrize("N,ab,gd", [(1, (0.1, -0.3), (0.5, 0.25)),
                                     (100, (0.1, -0.3), (-0.45, 0.3)),
                                     (1024, (-0.2, 0.4), (0.5, 0.5)),
                                     (3001, (0.3, 0.1), (-0.1, -0.4)),
                                     (16384, (-0.45, 0.3), (0.1, -0.3))])
def test_j2j_matches_oracle(lib, oracle_mod, N, ab, gd):
    import torch
    c = coeffs(N, N)
    src, dst = lib.cjt_plan(N, *ab), lib.cjt_plan(N, *gd)
    y = lib.jacobi_to_jacobi(src, dst, torch.as_tensor(c, device="cuda")).cpu().numpy()
    ref = oracle_mod.jacobi_to_jacobi(c, *ab, *gd, quad=N <= 4096)
    e = rel2(y, ref)
    print(f"N={N} {ab}->{gd}: {e:.2e}")
    assert e <= tol(N)


def test_j2j_same_parameters_round_trip(lib):
    import torch
    N = 5000
    c = coeffs(N, 3)
    p = lib.cjt_plan(N, 0.2, -0.1)
    y = lib.jacobi_to_jacobi(p, p, torch.as_tensor(c, device="cuda")).cpu().numpy()
    assert rel2(y, c) <= tol(N)


def test_j2j_batched_matches_single(lib):
    """Uneven batch: every slice equals the single call on the same plans
    (batch-invariant plans, so bitwise)."""
    import torch
    Ns = [64, 700, 4096, 9000, 2]
    rng = np.random.default_rng(11)
    src = [lib.cjt_plan(N, *rng.uniform(-0.5, 0.5, 2), 0, lib.CJT_BATCH_INVARIANT) for N in Ns]
    dst = [lib.cjt_plan(N, *rng.uniform(-0.5, 0.5, 2), 0, lib.CJT_BATCH_INVARIANT) for N in Ns]
    cs = [coeffs(N, 20 + i) for i, N in enumerate(Ns)]
    offs = np.concatenate([[0], np.cumsum([N + 1 for N in Ns])]).astype(np.int64)
    x = torch.as_tensor(np.concatenate(cs), device="cuda")
    y = torch.empty_like(x)
    lib.cjt_jacobi_to_jacobi_batched(src, dst, offs, x, y)
    yb = y.cpu().numpy()
    for i, N in enumerate(Ns):
        single = lib.jacobi_to_jacobi(src[i], dst[i], torch.as_tensor(cs[i], device="cuda")).cpu().numpy()
        assert np.array_equal(yb[offs[i]:offs[i + 1]], single), f"slice {i} (N={N})"


def test_j2j_fp32_bulk(lib, oracle_mod):
    import torch
    N = 8192
    c = coeffs(N, 5)
    f = lib.CJT_FP32_BULK
    src, dst = lib.cjt_plan(N, 0.1, -0.3, 0, f), lib.cjt_plan(N, 0.4, 0.2, 0, f)
    y = lib.jacobi_to_jacobi(src, dst, torch.as_tensor(c, device="cuda")).cpu().numpy()
    assert rel2(y, oracle_mod.jacobi_to_jacobi(c, 0.1, -0.3, 0.4, 0.2)) <= 1e-5


def test_j2j_argument_errors(lib):
    import torch
    x = torch.zeros(101, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    a, b = lib.cjt_plan(100, 0.1, 0.1), lib.cjt_plan(200, 0.1, 0.1)
    c32 = lib.cjt_plan(100, 0.1, 0.1, 0, lib.CJT_FP32_BULK)
    for args in ((a, b, x, y), (a, a, x, x), (a, c32, x, y)):
        with pytest.raises(lib.CJTError) as ei:
            lib.cjt_jacobi_to_jacobi(*args)
        assert ei.value.status == lib.CJT_EINVAL
    with pytest.raises(lib.CJTError) as ei:
        lib.cjt_jacobi_to_jacobi_batched([a], [b], [0, 101], x, y)
    assert ei.value.status == lib.CJT_EINVAL
