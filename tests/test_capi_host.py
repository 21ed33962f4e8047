"""Host-side checks of the HIP library (no GPU needed): exports, argument
validation, the partition of Sec. 2.2 against an independent mpmath
evaluation of the paper's criterion, and the Stirling-series table."""
import os
import re
import subprocess
import sys

import mpmath as mp
import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def lib():
    from paper_1602_02618_amd import cjt
    cjt.load()
    return cjt


def test_exports_match_header(lib):
    """Every function declared in include/cjt.h is exported by libcjt_hip.so."""
    hdr = open(os.path.join(ROOT, "include", "cjt.h")).read()
    decl = set(re.findall(r"^\s*(?:cjt_status|const char\*|int)\s+(cjt_\w+)\s*\(", hdr, re.M))
    assert {"cjt_plan", "cjt_forward", "cjt_inverse", "cjt_forward_batched", "cjt_inverse_batched"} <= decl
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(cjt_\w+)", out))
    assert decl <= exported, decl - exported
    assert set(lib._EXPORTS) == decl


@pytest.mark.parametrize("args,status", [
    (((1 << 21) + 1, 0.1, 0.1, 0), "CJT_EUNSUPPORTED"),
    ((0, 0.1, 0.1, 0), "CJT_EINVAL"),
    ((1024, 0.6, 0.1, 0), "CJT_EDOMAIN"),
    ((1024, -0.5, 0.1, 0), "CJT_EDOMAIN"),
    ((1024, 0.1, float("nan"), 0), "CJT_EDOMAIN"),
    ((1024, 0.1, 0.1, 1), "CJT_EDOMAIN"),
    ((1024, 0.1, 0.1, 31), "CJT_EDOMAIN"),
])
def test_argument_errors(lib, args, status):
    with pytest.raises(lib.CJTError) as e:
        lib.cjt_plan_describe(*args)
    assert e.value.status == getattr(lib, status)
    assert lib.cjt_last_error() != ""


def _mp_log_gM(theta, M, a, b):
    """log of the envelope g_M(theta) of Sec. 2.2, at 40 digits."""
    a, b = mp.mpf(a), mp.mpf(b)
    s, c = mp.sin(theta / 2), mp.cos(theta / 2)
    tot = mp.mpf(0)
    for l in range(M + 1):
        coef = mp.rf(0.5 + a, l) * mp.rf(0.5 - a, l) * mp.rf(0.5 + b, M - l) * mp.rf(0.5 - b, M - l) / (
            mp.factorial(l) * mp.factorial(M - l))
        tot += coef * c ** (l - M - b - 0.5) / s ** (l + a + 0.5)
    return mp.log(tot)


def _mp_log_2C(n, M, a, b):
    """log 2 C_{n,M} from eq. Cnmab with mpmath's Gamma."""
    a, b = mp.mpf(a), mp.mpf(b)
    return mp.log(2) + (2 * n - M + a + b + 1) * mp.log(2) + mp.log(mp.beta(n + a + 1, n + b + 1)) - mp.log(mp.pi) \
        - mp.log(mp.rf(2 * n + a + b + 2, M))


@pytest.mark.parametrize("N,a,b,M", [(1024, 0.1, -0.3, 12), (4096, -0.45, 0.3, 7), (65536, 0.37, 0.12, 13),
                                     (512, 0.5, -0.2, 9)])
def test_partition_matches_paper_criterion(lib, N, a, b, M):
    """Windows of every block satisfy 2 C_{j_k,M} g_M(theta_i) < eps inside and fail
    just outside (Sec. 2.2); blocks are nested, degree ranges tile [j_K, N]."""
    mp.mp.dps = 40
    info = lib.cjt_plan_describe(N, a, b, M)
    for part, G in ((info.fwd, N), (info.inv, 2 * N)):
        bl = part.blocks()
        assert part.nblocks >= 1
        # n_M (eq. for n_M, envelope at pi/2)
        lg = _mp_log_gM(mp.pi / 2, M, a, b)
        nM = int(mp.floor(mp.exp(-(mp.log(EPS) + (2 * M - 1) * mp.log(2) + mp.log(mp.pi) / 2 - lg) / (M + 0.5))))
        assert abs(part.n_M - nM) <= 1
        prev_hi = N + 1
        for k, (dlo, dhi, wlo, whi) in enumerate(bl):
            assert dhi == prev_hi and dlo < dhi
            prev_hi = dlo
            assert dlo > part.n_M
            l2c = _mp_log_2C(dlo, M, a, b)
            inside = lambda i: l2c + _mp_log_gM(mp.pi * i / G, M, a, b) < mp.log(EPS)
            assert inside(wlo) and inside(whi) and inside(part.theta_bar)
            if wlo > 1:
                assert not inside(wlo - 1)
            if whi < G - 1:
                assert not inside(whi + 1)
            if k > 0:
                assert bl[k - 1][2] <= wlo and whi <= bl[k - 1][3]
        # recurrence entries = sum over points of the degrees left to recurrence
        cut = np.full(G + 1, N + 1, dtype=np.int64)
        for (dlo, dhi, wlo, whi) in bl:
            cut[wlo:whi + 1] = dlo
        assert part.rec_entries == int(cut.sum())


def test_partition_alpha_K(lib):
    info = lib.cjt_plan_describe(65536, 0.1, -0.3, 12)
    p = info.fwd
    aN = min(1 / np.log(65536 / p.n_M), 0.5)
    assert abs(p.alpha_N - aN) < 1e-15
    assert p.K == int(np.ceil(np.log(65536 / p.n_M) / np.log(1 / aN)))
    # j_k = floor(alpha_N^k N)
    for k, (dlo, _, _, _) in enumerate(p.blocks(), start=1):
        assert dlo == int(np.floor(aN ** k * 65536))


def test_exact_one_term_case(lib):
    """a = b = 1/2: every f_m with m >= 1 vanishes, one term is exact."""
    info = lib.cjt_plan_describe(1024, 0.5, 0.5, 0)
    assert info.M == 1 and info.fwd.blocks() == [(2, 1025, 1, 1023)]


def test_auto_M_in_range(lib):
    for (a, b) in [(0.1, -0.3), (-0.49, 0.49), (0.3, 0.3)]:
        info = lib.cjt_plan_describe(65536, a, b, 0)
        assert 5 <= info.M <= 20


def test_stirling_table1_from_bound():
    """Table 1 follows from R_N(z) <= (1 + zeta(N)) Gamma(N) / ((2 pi)^(N+1) z^N) (Sec. 4.1):
    at each z_min, N terms suffice for R/S < eps/20, N-1 do not, and z_min - 1 is not enough."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1602_02618_amd", "csrc"))
    from gen_stirling import stirling_coefficients
    rows = [tuple(int(v) for v in l.split()) for l in open(os.path.join(ROOT, "tests", "golden", "stirling_table1.txt"))
            if l.strip() and not l.startswith("#")]
    mp.mp.dps = 40
    a = stirling_coefficients(20)
    lim = mp.mpf(EPS) / 20
    bound = lambda n, z: (1 + mp.zeta(n)) * mp.gamma(n) / ((2 * mp.pi) ** (n + 1) * mp.mpf(z) ** n)
    S = lambda n, z: mp.fsum(mp.mpf(a[k].numerator) / a[k].denominator / mp.mpf(z) ** k for k in range(n))
    assert len(rows) == 14
    for z, n in rows:
        assert bound(n, z) / S(n, z) < lim
        assert bound(n - 1, z) / S(n - 1, z) >= lim
        assert bound(n, z - 1) / S(n, z - 1) >= lim


def test_stirling_coefficients_match_gamma():
    """The generated a_n reproduce Gamma(z) / (sqrt(2 pi) z^(z-1/2) e^-z) at z = 30 to 1e-30."""
    sys.path.insert(0, os.path.join(ROOT, "paper_1602_02618_amd", "csrc"))
    from gen_stirling import stirling_coefficients
    mp.mp.dps = 50
    a = stirling_coefficients(17)
    z = mp.mpf(30)
    ref = mp.gamma(z) / (mp.sqrt(2 * mp.pi) * z ** (z - 0.5) * mp.exp(-z))
    ser = mp.fsum(mp.mpf(a[k].numerator) / a[k].denominator / z ** k for k in range(17))
    assert abs(ser / ref - 1) < 1e-22
    assert str(a[1]) == "1/12" and str(a[2]) == "1/288" and str(a[3]) == "-139/51840"


def test_schedule_table_host(lib, tmp_path):
    """The split table: validation, effect on plan descriptions (host only),
    save and load."""
    N = 65536  # forward FFT length 65536 = 2^16 (two passes), inverse 2^17
    d0 = lib.cjt_plan_describe(N, 0.1, 0.2)
    assert d0.fft_log2_cols_fwd == 8 and d0.fft_log2_cols_inv == 8  # default: floor(lg / 2)
    for bad in ((4096, 0, 0, 0, 6), (65536, 0, 0, 0, 3), (65536, 0, 0, 0, 13), (65537, 0, 0, 0, 8)):
        with pytest.raises(lib.CJTError) as e:
            lib.cjt_tune_set(*bad)
        assert e.value.status == lib.CJT_EINVAL
    try:
        lib.cjt_tune_set(65536, 0, 0, 0, 5)
        lib.cjt_tune_set(1 << 17, 1, 0, 0, 11)
        d1 = lib.cjt_plan_describe(N, 0.1, 0.2)
        assert d1.fft_log2_cols_fwd == 5 and d1.fft_log2_cols_inv == 11
        assert lib.cjt_plan_describe(N, 0.1, 0.2, 0, lib.CJT_FP32_BULK).fft_log2_cols_fwd == 8  # other precision
        path = str(tmp_path / "sched.txt")
        lib.cjt_tune_save(path)
        lines = [l.split() for l in open(path) if not l.startswith("#")]
        assert ["65536", "0", "0", "0", "5"] in lines and ["131072", "1", "0", "0", "11"] in lines
        lib.cjt_tune_set(65536, 0, 0, 0, -1)
        lib.cjt_tune_set(1 << 17, 1, 0, 0, -1)
        assert lib.cjt_plan_describe(N, 0.1, 0.2).fft_log2_cols_fwd == 8
        lib.cjt_tune_load(path)
        assert lib.cjt_plan_describe(N, 0.1, 0.2).fft_log2_cols_fwd == 5
        # chirp-z lengths are keyed by their convolution length: N = 70000 -> P = 2^18
        lib.cjt_tune_set(1 << 18, 0, 1, 0, 7)
        assert lib.cjt_plan_describe(70000, 0.1, 0.2).fft_log2_cols_fwd == 7
        bad = tmp_path / "bad.txt"
        bad.write_text("65536 0 0 0 99\n")
        with pytest.raises(lib.CJTError):
            lib.cjt_tune_load(str(bad))
    finally:
        for key in ((65536, 0, 0, 0), (1 << 17, 1, 0, 0), (1 << 18, 0, 1, 0)):
            lib.cjt_tune_set(*key, -1)


def test_jacobi_to_jacobi_null_arguments(lib):
    """Argument checks of the Jacobi-to-Jacobi entry points return before any
    device work: null plans or buffers are CJT_EINVAL, an empty batch is OK."""
    raw = lib.load()
    assert raw.cjt_jacobi_to_jacobi(None, None, None, None, None) == lib.CJT_EINVAL
    assert raw.cjt_jacobi_to_jacobi_batched(None, None, 1, None, None, None, None) == lib.CJT_EINVAL
    assert raw.cjt_jacobi_to_jacobi_batched(None, None, -1, None, None, None, None) == lib.CJT_EINVAL
    assert raw.cjt_jacobi_to_jacobi_batched(None, None, 0, None, None, None, None) == lib.CJT_OK


@pytest.mark.parametrize("a,b,sa,sb", [(1.3, 0.1, 1, 0), (-0.7, 2.4, -1, 2), (0.5, -0.5, 0, -1), (2.5, -0.95, 2, -1)])
def test_shift_split_on_the_host(lib, a, b, sa, sb):
    """CJT_SHIFT plans (Sec. 1.2 shifts): the core runs at (a - sa, b - sb) in
    (-1/2, 1/2]^2; the plan reports the caller's parameters and the shifts."""
    info = lib.cjt_plan_describe(1024, a, b, 0, lib.CJT_SHIFT)
    assert (info.shift_alpha, info.shift_beta) == (sa, sb)
    assert abs(info.alpha - a) < 1e-15 and abs(info.beta - b) < 1e-15
    base = lib.cjt_plan_describe(1024, a - sa, b - sb, 0)
    assert info.fwd.rec_entries == base.fwd.rec_entries and info.inv.nblocks == base.inv.nblocks


@pytest.mark.parametrize("a,b", [(2.6, 0.1), (-1.0, 0.0), (0.0, float("nan"))])
def test_shift_domain(lib, a, b):
    with pytest.raises(lib.CJTError) as e:
        lib.cjt_plan_describe(1024, a, b, 0, lib.CJT_SHIFT)
    assert e.value.status == lib.CJT_EDOMAIN
