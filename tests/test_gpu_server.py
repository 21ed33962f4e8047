"""Transform server (cjt_server_*): results against the oracle, bitwise
equality of a request served inside a mix with the same request run alone,
admission inside the device budget with plan eviction, cancellation, the
load generator and the error paths."""
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


def make_requests(lib, Ns, seed, repeat_first=True):
    """(flags, N, alpha, beta, coeffs) per request, both directions
    alternating; the first key repeats at the end to give a plan hit."""
    rng = np.random.default_rng(seed)
    reqs = []
    for i, N in enumerate(Ns):
        a, b = float(rng.uniform(-0.5, 0.5)), float(rng.uniform(-0.5, 0.5))
        d = lib.CJT_DIR_FWD if i % 2 == 0 else lib.CJT_DIR_INV
        reqs.append((d, N, a, b, inputs.decaying_coeffs(rng, N, 1.0)))
    if repeat_first:
        d, N, a, b, _ = reqs[0]
        reqs.append((d, N, a, b, inputs.decaying_coeffs(rng, N, 1.0)))
    return reqs


def serve(lib, reqs, paused, **cfg):
    """Runs the requests through a fresh server; returns outputs and stats."""
    import torch
    xs = [torch.as_tensor(r[4], device="cuda") for r in reqs]
    ys = [torch.full_like(x, float("nan")) for x in xs]
    torch.cuda.synchronize()
    with lib.cjt_server_create(start_paused=paused, **cfg) as srv:
        tickets = [srv.submit(d, N, a, b, x, y) for (d, N, a, b, _), x, y in zip(reqs, xs, ys)]
        if paused:
            lib.cjt_server_pause(srv, False)
        res = [srv.wait(t) for t in tickets]
        stats = srv.stats()
    return [y.cpu().numpy() for y in ys], res, stats


def alone(lib, reqs):
    """Each request on its own with a batch-invariant plan."""
    import torch
    outs = []
    for d, N, a, b, c in reqs:
        p = lib.cjt_plan(N, a, b, 0, lib.CJT_BATCH_INVARIANT)
        x = torch.as_tensor(c, device="cuda")
        y = lib.forward(p, x) if d == lib.CJT_DIR_FWD else lib.inverse(p, x)
        outs.append(y.cpu().numpy())
        p.destroy()
    return outs


MIX = [64, 100, 1024, 3001, 4096, 5000, 8192, 2, 777, 1, 12345, 65536]


def test_server_matches_oracle_and_alone(lib, oracle_mod):
    reqs = make_requests(lib, MIX, 31)
    budget = 4 << 30
    ya, ra, sa = serve(lib, reqs, True, hbm_budget=budget, max_batch=64)
    yb, rb, sb = serve(lib, reqs, False, hbm_budget=budget, max_batch=3)
    yc = alone(lib, reqs)
    print(f"paused start: {sa.batches} calls, mean batch {sa.mean_batch:.1f}; "
          f"max_batch 3: {sb.batches} calls, mean batch {sb.mean_batch:.1f}")
    for i, (d, N, a, b, c) in enumerate(reqs):
        assert ra[i][0] == lib.CJT_OK and rb[i][0] == lib.CJT_OK
        assert np.array_equal(ya[i], yc[i]), f"request {i} (N={N}) differs in a mix from alone"
        assert np.array_equal(yb[i], yc[i]), f"request {i} (N={N}) differs between batchings"
        if N <= 16384:
            fn = oracle_mod.forward if d == lib.CJT_DIR_FWD else oracle_mod.inverse
            e = rel2(ya[i], fn(c, a, b, quad=N <= 4096))
            print(f"  N={N} {'fwd' if d == lib.CJT_DIR_FWD else 'inv'} {e:.2e}")
            assert e <= tol(N)
    assert sa.completed == len(reqs) and sa.failed == 0
    assert sa.plan_hits >= 1 and sa.plan_misses == len(reqs) - 1
    assert sa.peak_used_bytes <= budget and sa.budget_bytes == budget


def test_server_evicts_within_budget(lib):
    """A budget that holds about three plans: later keys evict idle plans,
    usage never passes the budget, and results stay those of alone runs."""
    N = 4096
    arena = lib.cjt_plan_describe(N, 0.1, -0.2).device_bytes
    ws = 64 << 20
    fixed = ws + 2 * (16 << 20)  # workspace + two descriptor buffers of 16 MiB (max_batch 4)
    budget = fixed + 3 * arena + (2 << 20)
    reqs = make_requests(lib, [N] * 10, 32, repeat_first=False)
    y, r, s = serve(lib, reqs, False, hbm_budget=budget, workspace_bytes=ws, max_batch=4)
    ref = alone(lib, reqs)
    print(f"budget {budget / 2**20:.1f} MiB, plan {arena / 2**20:.2f} MiB: evictions {s.plan_evictions}, "
          f"stalls {s.admission_stalls}, peak {s.peak_used_bytes / 2**20:.1f} MiB")
    assert all(st == lib.CJT_OK for st, _ in r)
    for i in range(len(reqs)):
        assert np.array_equal(y[i], ref[i])
    assert s.plan_evictions >= 1
    assert s.peak_used_bytes <= budget
    assert s.plans_resident <= 3


def test_server_rejects_plan_over_budget(lib):
    """A plan larger than the whole heap fails with CJT_ENOMEM; requests that
    fit are served by the same server."""
    import torch
    ws = 64 << 20
    budget = ws + 2 * (16 << 20) + (3 << 20)
    big = torch.zeros(65537, dtype=torch.float64, device="cuda")
    small = torch.as_tensor(inputs.decaying_coeffs(np.random.default_rng(1), 64, 1.0), device="cuda")
    yb, ys = torch.empty_like(big), torch.empty_like(small)
    torch.cuda.synchronize()
    with lib.cjt_server_create(budget, workspace_bytes=ws, max_batch=4) as srv:
        t1 = srv.submit(lib.CJT_DIR_FWD, 65536, 0.1, 0.2, big, yb)
        t2 = srv.submit(lib.CJT_DIR_FWD, 64, 0.1, 0.2, small, ys)
        assert srv.wait(t1)[0] == lib.CJT_ENOMEM
        assert srv.wait(t2)[0] == lib.CJT_OK
        s = srv.stats()
    assert s.failed == 1 and s.completed == 1


def test_server_cancel_pause_drain(lib):
    import torch
    reqs = make_requests(lib, [100, 200, 300], 33, repeat_first=False)
    xs = [torch.as_tensor(r[4], device="cuda") for r in reqs]
    ys = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    with lib.cjt_server_create(1 << 30, start_paused=True) as srv:
        t = [srv.submit(d, N, a, b, x, y) for (d, N, a, b, _), x, y in zip(reqs, xs, ys)]
        assert lib.cjt_server_cancel(srv, t[1]) == lib.CJT_OK
        with pytest.raises(lib.CJTError) as ei:
            lib.cjt_server_drain(srv)  # paused with requests queued
        assert ei.value.status == lib.CJT_EBUSY
        lib.cjt_server_pause(srv, False)
        lib.cjt_server_drain(srv)
        assert lib.cjt_server_cancel(srv, t[0]) == lib.CJT_EBUSY  # already served
        assert srv.wait(t[1])[0] == lib.CJT_ECANCELED
        assert srv.wait(t[0])[0] == lib.CJT_OK and srv.wait(t[2])[0] == lib.CJT_OK
        assert lib.cjt_server_cancel(srv, t[0]) == lib.CJT_EINVAL  # forgotten after wait
        s = srv.stats(reset=True)
        assert s.cancelled == 1 and s.completed == 2
        assert srv.stats().completed == 0


def test_server_argument_errors(lib):
    import torch
    x = torch.zeros(11, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(lib.CJTError) as ei:
        lib.cjt_server_create(1 << 20)  # cannot hold workspace and descriptor buffers
    assert ei.value.status == lib.CJT_EINVAL
    with lib.cjt_server_create(1 << 30) as srv:
        for args, code in (((lib.CJT_DIR_FWD | lib.CJT_DIR_INV, 10, 0.0, 0.0, x, y), lib.CJT_EINVAL),
                           ((lib.CJT_BATCH_INVARIANT | lib.CJT_DIR_FWD, 10, 0.0, 0.0, x, y), lib.CJT_EINVAL),
                           ((lib.CJT_DIR_FWD, 10, 0.7, 0.0, x, y), lib.CJT_EDOMAIN),
                           ((lib.CJT_DIR_FWD, 0, 0.0, 0.0, x, y), lib.CJT_EINVAL),
                           ((lib.CJT_DIR_FWD, 10, 0.0, 0.0, x, x), lib.CJT_EINVAL)):
            with pytest.raises(lib.CJTError) as ei:
                srv.submit(*args)
            assert ei.value.status == code
        with pytest.raises(lib.CJTError):
            srv.wait(12345)
        assert srv.stats().submitted == 0


def test_server_replay_poisson(lib, oracle_mod):
    """The load generator: Poisson arrivals, both precisions, keys from a
    small pool; every request completes with a positive latency and FP64
    results match the alone runs bitwise."""
    import torch
    rng = np.random.default_rng(34)
    pool = [(int(N), float(a), float(b)) for N, a, b in
            zip(np.exp(rng.uniform(np.log(128), np.log(8192), 8)).astype(int),
                rng.uniform(-0.5, 0.5, 8), rng.uniform(-0.5, 0.5, 8))]
    n = 200
    keys = rng.integers(0, len(pool), n)
    dirs = np.where(rng.random(n) < 0.5, lib.CJT_DIR_FWD, lib.CJT_DIR_INV)
    prec = np.where(rng.random(n) < 0.25, lib.CJT_FP32_BULK, 0)
    arrivals = np.cumsum(rng.exponential(200.0, n))  # mean 200 us apart
    reqs = [(int(dirs[i]), *pool[keys[i]], inputs.decaying_coeffs(rng, pool[keys[i]][0], 1.0)) for i in range(n)]
    xs = [torch.as_tensor(r[4], device="cuda") for r in reqs]
    ys = [torch.empty_like(x) for x in xs]
    torch.cuda.synchronize()
    with lib.cjt_server_create(2 << 30) as srv:
        tickets = lib.cjt_server_replay(srv, [r[0] | int(prec[i]) for i, r in enumerate(reqs)],
                                        [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs],
                                        xs, ys, arrivals)
        res = [srv.wait(t) for t in tickets]
        s = srv.stats()
    print(f"replay: {s.batches} calls, mean batch {s.mean_batch:.2f}, hits {s.plan_hits}, misses {s.plan_misses}, "
          f"p50 {s.lat_p50_us:.0f} us, p99 {s.lat_p99_us:.0f} us")
    assert all(st == lib.CJT_OK and lat > 0 for st, lat in res)
    assert s.completed == n and s.lat_count == n and s.plan_misses <= 2 * len(pool)
    fp64 = [i for i in range(n) if prec[i] == 0][:12]
    ref = alone(lib, [reqs[i] for i in fp64])
    for j, i in enumerate(fp64):
        assert np.array_equal(ys[i].cpu().numpy(), ref[j])
    for i in [i for i in range(n) if prec[i] != 0][:4]:
        d, N, a, b, c = reqs[i]
        fn = oracle_mod.forward if d == lib.CJT_DIR_FWD else oracle_mod.inverse
        assert rel2(ys[i].cpu().numpy(), fn(c, a, b, quad=N <= 4096)) <= 1e-5
