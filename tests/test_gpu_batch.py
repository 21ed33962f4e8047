"""Persistent batches (cjt_batch_*): uneven degrees in one launch sequence,
parity with the oracle and with the one-shot entry points, and HIP-graph
capture and replay."""
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


def make_batch(lib, Ns, seed, flags=0):
    import torch
    rng = np.random.default_rng(seed)
    params = [(float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5))) for _ in Ns]
    cs = [inputs.decaying_coeffs(rng, N, 1.0) for N in Ns]
    plans = [lib.cjt_plan(N, a, b, 0, flags) for N, (a, b) in zip(Ns, params)]
    offs = np.concatenate([[0], np.cumsum([N + 1 for N in Ns])]).astype(np.int64)
    x = torch.as_tensor(np.concatenate(cs), device="cuda")
    return params, cs, plans, offs, x


# every kernel family: power-of-two single pass, chirp-z single pass, two-pass
# power of two, two-pass chirp-z; tiny degrees without Hahn blocks
MIXED = [64, 100, 1024, 3001, 4096, 5000, 8192, 2, 777]


@pytest.mark.parametrize("direction", ["fwd", "inv"])
def test_batch_matches_oracle(lib, oracle_mod, direction):
    import torch
    params, cs, plans, offs, x = make_batch(lib, MIXED, 21)
    flag = lib.CJT_DIR_FWD if direction == "fwd" else lib.CJT_DIR_INV
    b = lib.cjt_batch_create(plans, offs, flag)
    info = b.info
    print(f"batch: {info.count} transforms, {info.launches} launches, {info.items} items, "
          f"{info.workspace_bytes / 2**20:.1f} MiB workspace")
    y = torch.empty_like(x)
    lib.cjt_batch_execute(b, x, y)
    y = y.cpu().numpy()
    for i, N in enumerate(MIXED):
        a, bb = params[i]
        quad = N <= 4096
        ref = (oracle_mod.forward if direction == "fwd" else oracle_mod.inverse)(cs[i], a, bb, quad=quad)
        e = rel2(y[offs[i]:offs[i + 1]], ref)
        print(f"  N={N} {direction} {e:.2e}")
        assert e <= tol(N)


def test_batch_equals_one_shot(lib):
    """The persistent batch and cjt_*_batched run the same kernels on the same
    items: results are bitwise equal."""
    import torch
    params, cs, plans, offs, x = make_batch(lib, MIXED, 22)
    for flag, fn in ((lib.CJT_DIR_FWD, lib.cjt_forward_batched), (lib.CJT_DIR_INV, lib.cjt_inverse_batched)):
        b = lib.cjt_batch_create(plans, offs, flag)
        y1 = torch.empty_like(x)
        y2 = torch.empty_like(x)
        lib.cjt_batch_execute(b, x, y1)
        fn(plans, offs, x, y2)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2)


@pytest.mark.parametrize("direction", ["fwd", "inv"])
def test_batch_graph_replay(lib, direction):
    """cjt_batch_execute captured into a HIP graph; every replay (with eager
    work and synchronisations in between, and new input values) matches an
    eager execution bitwise."""
    import torch
    params, cs, plans, offs, x = make_batch(lib, MIXED, 23)
    flag = lib.CJT_DIR_FWD if direction == "fwd" else lib.CJT_DIR_INV
    b = lib.cjt_batch_create(plans, offs, flag)
    y = torch.empty_like(x)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        lib.cjt_batch_execute(b, x, y)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        lib.cjt_batch_execute(b, x, y)
    ref = torch.empty_like(x)
    rng = np.random.default_rng(5)
    for rep in range(4):
        x.copy_(torch.as_tensor(rng.standard_normal(x.numel()) / np.arange(1, x.numel() + 1), device="cuda"))
        y.zero_()
        g.replay()
        torch.cuda.synchronize()
        lib.cjt_batch_execute(b, x, ref)  # eager, same input
        _ = (x * 2.0).sum().item()        # unrelated eager work between replays
        torch.cuda.synchronize()
        print(f"replay {rep}: max |diff| {float((y - ref).abs().max()):.3e}")
        assert torch.equal(y, ref)


def test_batch_errors(lib):
    import torch
    p = lib.cjt_plan(64, 0.1, 0.1)
    with pytest.raises(lib.CJTError) as e:
        lib.cjt_batch_create([p], [0, 64], lib.CJT_DIR_FWD)  # wrong offsets
    assert e.value.status == lib.CJT_EINVAL
    with pytest.raises(lib.CJTError) as e:
        lib.cjt_batch_create([p], [0, 65], 0)  # no direction
    assert e.value.status == lib.CJT_EINVAL
    b = lib.cjt_batch_create([p], [0, 65], lib.CJT_DIR_FWD)
    x = torch.zeros(65, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.CJTError) as e:
        lib.cjt_batch_execute(b, x, x)
    assert e.value.status == lib.CJT_EINVAL


def test_job_parallel_and_fused_agree(lib):
    """Calls of at most 64 instances spread each instance's Hahn jobs over
    workgroups (per-job parts added by a reduce in job order); larger calls add
    the jobs inside one workgroup.  Both round the same way: a call of 70
    instances equals each instance run alone, bitwise, in both directions
    (batch-invariant plans; power-of-two two-pass, single-workgroup and chirp-z
    lengths)."""
    import torch
    rng = np.random.default_rng(24)
    Ns = [8192, 1000, 5000, 16384, 65536, 300] + list(rng.integers(64, 3000, 64))
    plans = [lib.cjt_plan(int(N), *rng.uniform(-0.5, 0.5, 2), 0, lib.CJT_BATCH_INVARIANT) for N in Ns]
    cs = [rng.standard_normal(int(N) + 1) / (np.arange(int(N) + 1) + 1.0) for N in Ns]
    offs = np.concatenate([[0], np.cumsum([int(N) + 1 for N in Ns])]).astype(np.int64)
    x = torch.as_tensor(np.concatenate(cs), device="cuda")
    for fn, single in ((lib.cjt_forward_batched, lib.forward), (lib.cjt_inverse_batched, lib.inverse)):
        y = torch.empty_like(x)
        fn(plans, offs, x, y)
        yb = y.cpu().numpy()
        for i in range(6):
            ys = single(plans[i], torch.as_tensor(cs[i], device="cuda")).cpu().numpy()
            assert np.array_equal(yb[offs[i]:offs[i + 1]], ys), (fn.__name__, i, Ns[i])
