"""Parameters outside (-1/2, 1/2]^2 through integer shifts (CJT_SHIFT, Sec.
1.2) against the oracle, through the C-ABI.

Forward: the oracle's forward is the definition for any alpha, beta > -1; the
bound is the core's tolerance times 4 (the lowering of the input is a stable
backward recurrence).  Inverse: the problem's conditioning grows like N^s for
s unit shifts up, so the bound is the core's tolerance times the condition
number kappa measured on the same data with the oracle (relative output change
over relative input change for a random 1e-8 perturbation)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def tol(N):
    return 1e-13 * max(math.log2(N), 1.0)


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


def coeffs(N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0)


def kappa(oracle_mod, cheb, a, b, seed=0):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(cheb.size) * 1e-8 * np.linalg.norm(cheb) / math.sqrt(cheb.size)
    y0 = oracle_mod.inverse_shifted(cheb, a, b)
    y1 = oracle_mod.inverse_shifted(cheb + d, a, b)
    return (np.linalg.norm(y1 - y0) / np.linalg.norm(y0)) / (np.linalg.norm(d) / np.linalg.norm(cheb))


CASES = [(1, (1.3, -0.8)), (50, (-0.7, 2.4)), (1024, (0.5, -0.5)), (1024, (2.5, 1.1)),
         (4096, (-0.9, -0.95)), (4097, (1.6, 0.2)), (16384, (0.7, 1.5))]


@pytest.mark.parametrize("N,ab", CASES)
def test_shifted_forward_and_inverse_match_oracle(lib, oracle_mod, N, ab):
    import torch
    a, b = ab
    c = coeffs(N, N)
    p = lib.cjt_plan(N, a, b, 0, lib.CJT_SHIFT)
    info = p.info
    assert (info.shift_alpha, info.shift_beta) == (math.ceil(a - 0.5), math.ceil(b - 0.5))
    assert abs(info.alpha - a) < 1e-15 and abs(info.beta - b) < 1e-15
    x = torch.as_tensor(c, device="cuda")
    f = lib.forward(p, x).cpu().numpy()
    quad = N <= 4096
    fr = oracle_mod.forward(c, a, b, quad=quad)
    ef = rel2(f, fr)
    g = lib.inverse(p, torch.as_tensor(fr, device="cuda")).cpu().numpy()
    gr = oracle_mod.inverse_shifted(fr, a, b, quad=quad)
    k = kappa(oracle_mod, fr, a, b) if N <= 4097 else None
    ei = rel2(g, gr)
    print(f"N={N} {ab}: forward {ef:.2e}, inverse {ei:.2e}, kappa {k}")
    assert ef <= 4 * tol(N)
    if k is not None:
        assert ei <= 2 * tol(N) * max(1.0, k)
    else:
        assert ei <= 1e-9


def test_shifted_in_a_mixed_batch(lib):
    """Shifted and unshifted plans in one batched call: each slice equals
    the single call (batch-invariant plans, so bitwise), both directions."""
    import torch
    specs = [(300, 0.1, 0.2, 0), (1000, 1.4, -0.6, lib.CJT_SHIFT), (64, -0.3, 0.4, 0), (2049, -0.8, 2.2, lib.CJT_SHIFT)]
    plans = [lib.cjt_plan(N, a, b, 0, fl | lib.CJT_BATCH_INVARIANT) for N, a, b, fl in specs]
    cs = [coeffs(N, 40 + i) for i, (N, _, _, _) in enumerate(specs)]
    offs = np.concatenate([[0], np.cumsum([s[0] + 1 for s in specs])]).astype(np.int64)
    x = torch.as_tensor(np.concatenate(cs), device="cuda")
    x_keep = x.clone()
    for fn, single in ((lib.cjt_forward_batched, lib.forward), (lib.cjt_inverse_batched, lib.inverse)):
        y = torch.empty_like(x)
        fn(plans, offs, x, y)
        assert torch.equal(x, x_keep), "the input must not change"
        yb = y.cpu().numpy()
        for i in range(len(specs)):
            ys = single(plans[i], torch.as_tensor(cs[i], device="cuda")).cpu().numpy()
            assert np.array_equal(yb[offs[i]:offs[i + 1]], ys), (fn.__name__, i)


def test_shifted_jacobi_to_jacobi(lib, oracle_mod):
    """Coefficients decaying like (n+1)^-2: P_n^(1.5,.)(1) grows like n^1.5,
    so with (n+1)^-1 decay the function reaches O(N) at x = 1 and the core
    inverse's quadrature sum loses relative accuracy in proportion (measured:
    2e-11 at N = 2000 in the base family), a property of such inputs, not of
    the shifts."""
    import torch
    N = 2000
    c = np.random.default_rng(9).standard_normal(N + 1) / (np.arange(N + 1) + 1.0) ** 2
    src = lib.cjt_plan(N, 1.5, 0.5, 0, lib.CJT_SHIFT)
    dst = lib.cjt_plan(N, -0.7, 2.0, 0, lib.CJT_SHIFT)
    y = lib.jacobi_to_jacobi(src, dst, torch.as_tensor(c, device="cuda")).cpu().numpy()
    cheb = oracle_mod.forward(c, 1.5, 0.5, quad=True)
    ref = oracle_mod.inverse_shifted(cheb, -0.7, 2.0, quad=True)
    k = kappa(oracle_mod, cheb, -0.7, 2.0)
    assert rel2(y, ref) <= 4 * tol(N) * max(1.0, k)


def test_shift_argument_errors(lib):
    for args, code in (((100, 1.3, 0.1, 0, 0), lib.CJT_EDOMAIN),
                       ((100, 2.6, 0.1, 0, lib.CJT_SHIFT), lib.CJT_EDOMAIN),
                       ((100, -1.0, 0.1, 0, lib.CJT_SHIFT), lib.CJT_EDOMAIN),
                       ((100, 0.1, float("inf"), 0, lib.CJT_SHIFT), lib.CJT_EDOMAIN)):
        with pytest.raises(lib.CJTError) as ei:
            lib.cjt_plan(*args)
        assert ei.value.status == code
    p = lib.cjt_plan(100, 1.3, 0.1, 0, lib.CJT_SHIFT)
    with pytest.raises(lib.CJTError) as ei:
        lib.cjt_batch_create([p], [0, 101], lib.CJT_DIR_FWD)
    assert ei.value.status == lib.CJT_EUNSUPPORTED
