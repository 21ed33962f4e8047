"""Schedule autotuner: every accepted two-pass split gives the transform
within the FP64 tolerance of the default schedule (and of the oracle), the
tuner keeps the fastest split, and later plans use it."""
import math

import numpy as np
import pytest

from paper_1602_02618_amd import inputs

pytestmark = pytest.mark.gpu


def tol(N):
    return 1e-13 * max(math.log2(N), 1.0)


def rel2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1602_02618_amd import cjt
    cjt.load()
    return cjt


def split_keys(N):
    """(F, inverse, chirp, lo, hi) of the two-pass FFTs of degree N."""
    out = []
    for inv, L in ((0, N), (1, 2 * N)):
        if L & (L - 1) == 0:
            F, chirp = L, 0
        else:
            F, chirp = 1 << (2 * L - 2).bit_length(), 1
        if F <= 4096:
            continue
        lg = F.bit_length() - 1
        out.append((F, inv, chirp, max(4, lg - 11), min(11, lg - 4)))
    return out


def run(lib, N, a, b, c):
    import torch
    p = lib.cjt_plan(N, a, b)
    x = torch.as_tensor(c, device="cuda")
    f = lib.forward(p, x).cpu().numpy()
    g = lib.inverse(p, x).cpu().numpy()
    info = p.info
    return f, g, (info.fft_log2_cols_fwd, info.fft_log2_cols_inv)


@pytest.mark.parametrize("N", [8192, 70000])
def test_every_split(lib, oracle_mod, N):
    rng = np.random.default_rng(N + 3)
    a, b = float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5))
    c = inputs.decaying_coeffs(rng, N, 1.0)
    f0, g0, _ = run(lib, N, a, b, c)
    if N <= 8192:
        assert rel2(f0, oracle_mod.forward(c, a, b)) <= tol(N)
        assert rel2(g0, oracle_mod.inverse(c, a, b)) <= tol(N)
    keys = split_keys(N)
    try:
        for F, inv, chirp, lo, hi in keys:
            for lg1 in range(lo, hi + 1):
                lib.cjt_tune_set(F, inv, chirp, 0, lg1)
                f, g, cols = run(lib, N, a, b, c)
                assert cols[inv] == lg1
                ef, eg = rel2(f, f0), rel2(g, g0)
                print(f"N={N} F={F} {'inv' if inv else 'fwd'} lg1={lg1}: fwd {ef:.1e} inv {eg:.1e}")
                assert ef <= tol(N) and eg <= tol(N)
            lib.cjt_tune_set(F, inv, chirp, 0, -1)
    finally:
        for F, inv, chirp, _, _ in keys:
            lib.cjt_tune_set(F, inv, chirp, 0, -1)


def test_autotune_keeps_fastest(lib, tmp_path):
    N = 65536
    try:
        ents = lib.cjt_autotune(N, lib.CJT_FP64, batch=4, reps=2)
        assert [(e.fft_len, e.inverse) for e in ents] == [(N, 0), (2 * N, 1)]
        for e in ents:
            print(e.as_dict())
            assert e.candidates >= 3 and e.ms_best <= e.ms_default and e.ms_best > 0
        info = lib.cjt_plan(N, 0.2, -0.1).info
        assert (info.fft_log2_cols_fwd, info.fft_log2_cols_inv) == (ents[0].log2_cols_best, ents[1].log2_cols_best)
        path = str(tmp_path / "tuned.txt")
        lib.cjt_tune_save(path)
        assert len([l for l in open(path) if not l.startswith("#")]) >= 2
    finally:
        lib.cjt_tune_set(N, 0, 0, 0, -1)
        lib.cjt_tune_set(2 * N, 1, 0, 0, -1)
