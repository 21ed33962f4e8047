"""Benchmark: batched forward + inverse Chebyshev--Jacobi transforms on one MI355X.

Workload (default): 256 independent transforms at N = 65536 with
(alpha, beta) ~ U(-1/2, 1/2)^2 per instance and c_n = z_n / (n+1), z ~ N(0,1)
(seeded, synthetic; the paper's experiments use the same kind of inputs).
One step = one batched forward transform of all 256 coefficient vectors
followed by one batched inverse transform of its output.  Inputs, outputs and
plans are resident in HBM before timing starts; plans are built once.

Prints one JSON line.  `value` is coefficients/s of the FP64 path,
2 * 256 * (N+1) per step; the FP32-bulk path (FP32 DCT-I/DST-I in the Hahn
blocks) is reported beside it.  `roofline` covers the kernel with the largest
share of the FP64 step, timed with HIP events on its own stream over the timed
steps; `cpu_baseline` times the CPU oracle on one instance (forward + inverse).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 vector
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--count", type=int, default=256, help="transforms per batch")
    ap.add_argument("--N", type=int, default=65536)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the latency (N=1024), N=2^20 and uneven-batch (4096 instances) measurements")
    ap.add_argument("--autotune", action="store_true",
                    help="tune the two-pass FFT splits for this batch before planning (schedule only)")
    ap.add_argument("--pmc-calibration", action="store_true",
                    help="after timing, copy 256 MiB on the device (the counter calibration of the traffic summary)")
    ap.add_argument("--workload", choices=("batch", "serve"), default="batch",
                    help="batch: 256 x N=65536 forward+inverse (default); serve: the request stream")
    ap.add_argument("--serve-requests", type=int, default=20000, help="requests per measured rate")
    ap.add_argument("--serve-warmup", type=int, default=1000)
    ap.add_argument("--serve-capacity", type=int, default=3000, help="requests of the saturating burst")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-max-batch", type=int, default=256)
    ap.add_argument("--serve-streams", default="pool,continuous")
    ap.add_argument("--serve-precisions", default="fp64,fp32_bulk")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_steps(torch, step, steps, warmup):
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in evs])  # ms
    return wall, per


SERVE_NMAX = 1 << 18


def serve_main(args):
    """Serving stream: Poisson arrivals of forward/inverse requests (50/50),
    N log-uniform in [128, 2^18], (alpha, beta) ~ U(-1/2, 1/2)^2, through the
    continuous-batching server.  For each key stream (a pool of 256 keys drawn
    once, and continuous keys) and each path (FP64, FP32-bulk): the saturated
    capacity C from a burst, then Poisson runs at 0.5 C and 0.8 C."""
    import torch
    from paper_1602_02618_amd import cjt, inputs

    torch.cuda.set_device(0)
    cjt.load()
    rng = np.random.default_rng(args.seed)
    n_in, ring = 16, 2048
    X = torch.as_tensor(np.stack([inputs.decaying_coeffs(rng, SERVE_NMAX, 1.0) for _ in range(n_in)]),
                        device="cuda")
    Y = torch.empty((ring, SERVE_NMAX + 1), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    in_ptr = [X[i].data_ptr() for i in range(n_in)]
    out_ptr = [Y[i].data_ptr() for i in range(ring)]
    budget = int(args.serve_budget_gb * (1 << 30))
    precs = {"fp64": 0, "fp32_bulk": cjt.CJT_FP32_BULK}
    streams = [s for s in args.serve_streams.split(",") if s]
    result = {}
    base = [0]

    def replay(srv, req, lo, hi, arrivals, prec):
        fwd, Ns, al, be = req
        idx = range(lo, hi)
        flags = [(cjt.CJT_DIR_FWD if fwd[i] else cjt.CJT_DIR_INV) | prec for i in idx]
        d_in = [in_ptr[i % n_in] for i in idx]
        d_out = [out_ptr[(base[0] + j) % ring] for j in range(hi - lo)]
        base[0] += hi - lo
        tickets = cjt.cjt_server_replay(srv, flags, Ns[lo:hi], al[lo:hi], be[lo:hi], d_in, d_out, arrivals)
        res = [srv.wait(t) for t in tickets]
        bad = [st for st, _ in res if st != cjt.CJT_OK]
        if bad:
            raise RuntimeError(f"{len(bad)} requests failed, first status {bad[0]}")
        done = np.asarray(arrivals) + np.array([lat for _, lat in res])
        return float(done.max() - np.min(arrivals)) * 1e-6  # seconds from first arrival to last completion

    for sname in streams:
        pool = 256 if sname == "pool" else 0
        total = args.serve_warmup + args.serve_capacity + 2 * args.serve_requests
        req = inputs.serving_requests(total, args.seed + (1 if pool else 2), key_pool=pool)
        for pname in [p for p in args.serve_precisions.split(",") if p]:
            prec = precs[pname]
            rec = {}
            with cjt.cjt_server_create(budget, max_batch=args.serve_max_batch) as srv:
                pos = 0
                w = args.serve_warmup
                replay(srv, req, pos, pos + w, np.zeros(w), prec)
                pos += w
                srv.stats(reset=True)
                n = args.serve_capacity
                span = replay(srv, req, pos, pos + n, np.zeros(n), prec)
                pos += n
                st = srv.stats(reset=True)
                C = n / span
                rec["capacity_req_s"] = C
                rec["capacity_batch_mean"] = st.mean_batch
                log(f"serve {sname}/{pname}: capacity {C:.0f} req/s (burst of {n}, mean batch {st.mean_batch:.1f}, "
                    f"hits {st.plan_hits} misses {st.plan_misses})")
                for frac in (0.5, 0.8):
                    n = args.serve_requests
                    rate = frac * C
                    arr = inputs.poisson_arrivals(n, rate, args.seed + int(frac * 10))
                    span = replay(srv, req, pos, pos + n, arr, prec)
                    pos += n
                    st = srv.stats(reset=True)
                    hit = st.plan_hits / max(st.plan_hits + st.plan_misses, 1)
                    rec[f"{frac}C"] = {"rate_req_s": rate, "requests": n, "throughput_req_s": n / span,
                                       "p50_us": st.lat_p50_us, "p99_us": st.lat_p99_us, "mean_us": st.lat_mean_us,
                                       "max_us": st.lat_max_us, "mean_batch": st.mean_batch, "plan_hit_rate": hit,
                                       "plan_evictions": st.plan_evictions, "admission_stalls": st.admission_stalls,
                                       "peak_used_GiB": st.peak_used_bytes / 2**30}
                    log(f"  {frac}C = {rate:.0f} req/s: {n / span:.0f} req/s served, p50 {st.lat_p50_us:.0f} us, "
                        f"p99 {st.lat_p99_us:.0f} us, mean batch {st.mean_batch:.1f}, hit rate {hit:.3f}, "
                        f"evictions {st.plan_evictions}, peak {st.peak_used_bytes / 2**30:.1f} GiB")
            result[f"{sname}/{pname}"] = rec
    # FP32-bulk against the FP64 path on the same requests (pool keys)
    acc = None
    if "fp32_bulk" in args.serve_precisions and "fp64" in args.serve_precisions:
        req = inputs.serving_requests(64, args.seed + 7, key_pool=256)
        outs = {}
        for pname in ("fp64", "fp32_bulk"):
            base[0] = 0
            with cjt.cjt_server_create(budget, max_batch=args.serve_max_batch) as srv:
                replay(srv, req, 0, 64, np.zeros(64), precs[pname])
            outs[pname] = [Y[i, : int(req[1][i]) + 1].cpu().numpy() for i in range(64)]
        errs = [float(np.linalg.norm(outs["fp32_bulk"][i] - outs["fp64"][i]) / np.linalg.norm(outs["fp64"][i]))
                for i in range(64)]
        acc = {"requests": 64, "max_rel2": max(errs), "median_rel2": float(np.median(errs))}
        log(f"fp32-bulk vs fp64 path on 64 requests: max rel-2 {acc['max_rel2']:.2e}")
    head = result.get("pool/fp64", next(iter(result.values())))
    out = {
        "metric": "CJT serving: requests/s and p50/p99 latency (arrival to completion) at 0.5C and 0.8C",
        "value": head["0.8C"]["throughput_req_s"],
        "unit": "requests/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "Poisson request stream, forward/inverse 50/50, N log-uniform in [128, 2^18], "
                               "(alpha,beta)~U(-1/2,1/2)^2, c_n=randn/(n+1); key streams: pool of 256 keys, "
                               "continuous keys", "budget_GiB": args.serve_budget_gb,
                   "max_batch": args.serve_max_batch, "requests_per_rate": args.serve_requests,
                   "seed": args.seed},
        "streams": result,
        "fp32_bulk_vs_fp64": acc,
    }
    print(json.dumps(out))


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "hahn_inv_cols_batch256_N65536_traffic.md")


def event_ms(torch, fn, reps, warm):
    """Median and p99 of reps calls of fn, each bracketed by events on the current stream."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    t = np.array([a.elapsed_time(b) for a, b in evs])
    return float(np.median(t)), float(np.percentile(t, 99))


def extra_workloads(torch, cjt, inputs, seed):
    """The single-transform latency (N = 1024), the large transform (N = 2^20) and
    the uneven batch of 4096 forward transforms replayed from a HIP graph."""
    out = {}
    inst = inputs.small_single(seed)
    p = cjt.cjt_plan(inst.N, inst.alpha, inst.beta)
    x = torch.as_tensor(inst.coeffs, device="cuda")
    f = torch.empty_like(x)
    g = torch.empty_like(x)
    fm, f99 = event_ms(torch, lambda: cjt.cjt_forward(p, x, f), 1000, 100)
    im, i99 = event_ms(torch, lambda: cjt.cjt_inverse(p, f, g), 1000, 100)
    out["latency_N1024"] = {"forward_p50_us": fm * 1e3, "forward_p99_us": f99 * 1e3,
                            "inverse_p50_us": im * 1e3, "inverse_p99_us": i99 * 1e3, "calls": 1000,
                            "round_trip_rel_error": float(np.linalg.norm(g.cpu().numpy() - inst.coeffs)
                                                          / np.linalg.norm(inst.coeffs))}
    log(f"N=1024 latency: forward p50 {fm * 1e3:.1f} us p99 {f99 * 1e3:.1f} us, inverse p50 {im * 1e3:.1f} us "
        f"p99 {i99 * 1e3:.1f} us")
    big = inputs.large_single(seed)
    pb = cjt.cjt_plan(big.N, big.alpha, big.beta)
    xb = torch.as_tensor(big.coeffs, device="cuda")
    fb = torch.empty_like(xb)
    gb = torch.empty_like(xb)
    fm, _ = event_ms(torch, lambda: cjt.cjt_forward(pb, xb, fb), 10, 2)
    im, _ = event_ms(torch, lambda: cjt.cjt_inverse(pb, fb, gb), 10, 2)
    info = pb.info
    out["large_N2^20"] = {"forward_ms": fm, "inverse_ms": im, "M": info.M, "blocks_fwd": info.fwd.nblocks,
                          "blocks_inv": info.inv.nblocks,
                          "round_trip_rel_error": float(np.linalg.norm(gb.cpu().numpy() - big.coeffs)
                                                        / np.linalg.norm(big.coeffs))}
    log(f"N=2^20: forward {fm:.2f} ms, inverse {im:.2f} ms (M={info.M})")
    insts = inputs.batch_log_uniform_N(4096, 64, 16384, seed, r=1.0)
    t0 = time.perf_counter()
    plans = [cjt.cjt_plan(i.N, i.alpha, i.beta) for i in insts]
    t_plan = time.perf_counter() - t0
    offs = np.concatenate([[0], np.cumsum([i.N + 1 for i in insts])]).astype(np.int64)
    xu = torch.as_tensor(np.concatenate([i.coeffs for i in insts]), device="cuda")
    yu = torch.empty_like(xu)
    batch = cjt.cjt_batch_create(plans, offs, cjt.CJT_DIR_FWD)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        cjt.cjt_batch_execute(batch, xu, yu)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        cjt.cjt_batch_execute(batch, xu, yu)
    gm, g99 = event_ms(torch, graph.replay, 100, 3)
    om, _ = event_ms(torch, lambda: cjt.cjt_forward_batched(plans, offs, xu, yu), 10, 2)
    coeffs = int(offs[-1])
    out["uneven_batch_4096"] = {"graph_replay_p50_ms": gm, "graph_replay_p99_ms": g99, "one_shot_ms": om,
                                "coefficients": coeffs, "coefficients_per_s": coeffs / (gm * 1e-3),
                                "plan_s": t_plan, "launches": batch.info.launches,
                                "workspace_GiB": batch.info.workspace_bytes / 2**30}
    log(f"uneven batch of 4096: graph replay p50 {gm:.2f} ms ({coeffs / (gm * 1e-3):.3e} coeff/s), one-shot "
        f"{om:.2f} ms, plans {t_plan:.1f} s")
    batch.destroy()
    out["jacobi_to_jacobi_256_N16384"] = jacobi_to_jacobi_workload(torch, cjt, inputs, seed)
    out["shifted_N65536"] = shifted_workload(torch, cjt, seed)
    return out


def shifted_workload(torch, cjt, seed):
    """One transform at N = 65536 with (alpha, beta) = (1.5, -0.7), outside
    (-1/2, 1/2]^2 (CJT_SHIFT: core at (0.5, 0.3), one unit of shift in each
    parameter), against the same N at the base parameters: the cost of the
    O(N) coefficient moves."""
    N = 65536
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(N + 1) / (np.arange(N + 1) + 1.0)
    ps = cjt.cjt_plan(N, 1.5, -0.7, 0, cjt.CJT_SHIFT)
    pb = cjt.cjt_plan(N, 0.5, 0.3)
    x = torch.as_tensor(c, device="cuda")
    f = torch.empty_like(x)
    g = torch.empty_like(x)
    r = {}
    for name, p in (("shifted", ps), ("base", pb)):
        fm, _ = event_ms(torch, lambda: cjt.cjt_forward(p, x, f), 20, 3)
        im, _ = event_ms(torch, lambda: cjt.cjt_inverse(p, f, g), 20, 3)
        r[name] = {"forward_ms": fm, "inverse_ms": im}
    cjt.cjt_forward(ps, x, f)
    cjt.cjt_inverse(ps, f, g)
    r["shifted"]["round_trip_rel_error"] = float(np.linalg.norm(g.cpu().numpy() - c) / np.linalg.norm(c))
    log(f"shifted N=65536 (1.5,-0.7): forward {r['shifted']['forward_ms']:.3f} ms, inverse "
        f"{r['shifted']['inverse_ms']:.3f} ms; base (0.5,0.3): forward {r['base']['forward_ms']:.3f} ms, inverse "
        f"{r['base']['inverse_ms']:.3f} ms; round trip {r['shifted']['round_trip_rel_error']:.2e}")
    return r


def jacobi_to_jacobi_workload(torch, cjt, inputs, seed):
    """256 Jacobi-to-Jacobi transforms at N = 16384, (a, b) -> (c, d) with all
    four parameters ~ U(-1/2, 1/2) per instance: one batched forward and one
    batched inverse through the library's Chebyshev buffer.  The accuracy
    figure is the relative 2-norm error of transforming back to (a, b); parity
    with the oracle is the tests' job."""
    count, N = 256, 16384
    src = inputs.batch_uniform_params(count, N, seed, r=1.0)
    dst = inputs.batch_uniform_params(count, N, seed + 1000, r=1.0)
    t0 = time.perf_counter()
    ps = [cjt.cjt_plan(i.N, i.alpha, i.beta) for i in src]
    pd = [cjt.cjt_plan(i.N, i.alpha, i.beta) for i in dst]
    t_plan = time.perf_counter() - t0
    offs = np.arange(count + 1, dtype=np.int64) * (N + 1)
    x = torch.as_tensor(np.concatenate([i.coeffs for i in src]), device="cuda")
    y = torch.empty_like(x)
    ms, m99 = event_ms(torch, lambda: cjt.cjt_jacobi_to_jacobi_batched(ps, pd, offs, x, y), 10, 2)
    back = torch.empty_like(x)
    cjt.cjt_jacobi_to_jacobi_batched(pd, ps, offs, y, back)
    xr = x.cpu().numpy()
    err = float(np.linalg.norm(back.cpu().numpy() - xr) / np.linalg.norm(xr))
    coeffs = count * (N + 1)
    log(f"Jacobi-to-Jacobi 256 x N=16384: {ms:.2f} ms ({coeffs / (ms * 1e-3):.3e} coeff/s), there-and-back rel-2 "
        f"{err:.2e}, plans {t_plan:.1f} s")
    return {"p50_ms": ms, "p99_ms": m99, "coefficients_per_s": coeffs / (ms * 1e-3),
            "there_and_back_rel_error": err, "plan_s": t_plan}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); independent transforms would shard "
              "across GPUs with no exchange, but no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    if args.workload == "serve":
        serve_main(args)
        return
    import torch
    from paper_1602_02618_amd import cjt, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    cjt.load()
    N, count = args.N, args.count
    insts = inputs.batch_uniform_params(count, N, args.seed, r=1.0)
    log(f"bench: {count} transforms at N={N}")

    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = [e.as_dict() for e in cjt.cjt_autotune(N, cjt.CJT_FP64, batch=count, reps=2)]
        if not args.no_fp32:
            tuned += [e.as_dict() for e in cjt.cjt_autotune(N, cjt.CJT_FP32_BULK, batch=count, reps=2)]
        log(f"autotune ({time.perf_counter() - t0:.1f} s): " +
            "; ".join(f"L={e['fft_len']} {'inv' if e['inverse'] else 'fwd'}{' fp32' if e['fp32'] else ''}: "
                      f"2^{e['log2_cols_default']} cols {e['ms_default']:.2f} ms -> 2^{e['log2_cols_best']} "
                      f"{e['ms_best']:.2f} ms" for e in tuned))
    t0 = time.perf_counter()
    plans64 = [cjt.cjt_plan(i.N, i.alpha, i.beta, 0, cjt.CJT_FP64) for i in insts]
    t_plan64 = time.perf_counter() - t0
    plans32 = []
    t_plan32 = 0.0
    if not args.no_fp32:
        t0 = time.perf_counter()
        plans32 = [cjt.cjt_plan(i.N, i.alpha, i.beta, 0, cjt.CJT_FP32_BULK) for i in insts]
        t_plan32 = time.perf_counter() - t0
    log(f"plans built: fp64 {t_plan64:.2f}s fp32-bulk {t_plan32:.2f}s")

    offs = np.concatenate([[0], np.cumsum([i.N + 1 for i in insts])]).astype(np.int64)
    x = torch.as_tensor(np.concatenate([i.coeffs for i in insts]), dtype=torch.float64, device="cuda")
    f = torch.empty_like(x)
    g = torch.empty_like(x)

    def make_step(plans):
        def step():
            cjt.cjt_forward_batched(plans, offs, x, f)
            cjt.cjt_inverse_batched(plans, offs, f, g)
        return step

    coeffs_per_step = 2 * int(offs[-1])
    results = {}
    for name, plans in (("fp64", plans64), ("fp32_bulk", plans32)):
        if not plans:
            continue
        step = make_step(plans)
        wall, per = time_steps(torch, step, args.steps, args.warmup)
        # kernel breakdown over a second timed pass of the same steps
        cjt.cjt_profile_enable(True)
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        cjt.cjt_profile_enable(False)
        kern = cjt.cjt_profile_collect()
        f_h = f[: offs[1]].cpu().numpy().copy()
        g_h = g[: offs[1]].cpu().numpy().copy()
        results[name] = dict(wall=wall, per=per, kern=kern, f0=f_h, g0=g_h)
        ms = wall / args.steps * 1e3
        log(f"{name}: {ms:.3f} ms/step, {coeffs_per_step / (wall / args.steps):.4e} coeff/s, "
            f"p50 {np.percentile(per, 50):.3f} ms p99 {np.percentile(per, 99):.3f} ms")
        for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["total_ms"]):
            log(f"   {k:28s} {v['total_ms'] / args.steps:8.3f} ms/step  "
                f"{v['flops'] / (v['total_ms'] * 1e-3) / 1e12 if v['total_ms'] > 0 else 0:7.2f} TFLOP/s alg")

    # FP32-bulk inverse on the FP64 forward output of instance 0 (same input as the FP64 inverse)
    err = {}
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        c0 = insts[0].coeffs
        threads = oracle.default_threads()
        t0 = time.perf_counter()
        f_ref = oracle.forward(c0, insts[0].alpha, insts[0].beta, threads=threads)
        g_ref = oracle.inverse(results["fp64"]["f0"], insts[0].alpha, insts[0].beta, threads=threads)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": 2 * (N + 1) / t_cpu, "unit": "coefficients/s", "cores": threads, "kind": "oracle",
               "sample": f"instance 0 of the batch: one forward and one inverse transform at N={N} "
                         f"(long double O(N^2) plain definition), {t_cpu:.1f} s"}
        rel = lambda a, b: float(np.linalg.norm(a - b) / np.linalg.norm(b))
        err["fp64_forward"] = rel(results["fp64"]["f0"], f_ref)
        err["fp64_inverse"] = rel(results["fp64"]["g0"], g_ref)
        if "fp32_bulk" in results:
            err["fp32_bulk_forward"] = rel(results["fp32_bulk"]["f0"], f_ref)
            fin = torch.as_tensor(results["fp64"]["f0"], dtype=torch.float64, device="cuda")
            g32 = cjt.inverse(plans32[0], fin).cpu().numpy()
            err["fp32_bulk_inverse"] = rel(g32, g_ref)
        err["tolerance_fp64"] = 1e-13 * math.log2(N)
        log(f"errors vs oracle (instance 0): {err}; oracle {t_cpu:.1f}s on {threads} threads")

    extra = None if args.no_extra else extra_workloads(torch, cjt, inputs, args.seed)
    if args.pmc_calibration:
        a = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    r64 = results["fp64"]
    t_step = r64["wall"] / args.steps
    kern = r64["kern"]
    top = max(kern.items(), key=lambda kv: kv[1]["total_ms"])
    tname, tv = top
    launches = max(tv["launches"], 1)
    t_launch = tv["total_ms"] * 1e-3 / launches                # average launch duration (s)
    alg_flops, alg_bytes = tv["flops"] / launches, tv["bytes"] / launches
    peak = PEAK_FP32_TFLOPS if tname.endswith("fp32") else PEAK_FP64_TFLOPS
    # the kernel's roofline: the larger of its compute and HBM time at peak
    alu_bound = alg_flops / (peak * 1e12) >= alg_bytes / (PEAK_HBM_GBS * 1e9)
    if alu_bound:
        achieved, unit, ceiling = alg_flops / t_launch / 1e12, "TFLOP/s", peak
    else:
        achieved, unit, ceiling = alg_bytes / t_launch / 1e9, "GB/s", PEAK_HBM_GBS
    from paper_1602_02618_amd import profiling
    rec = profiling.read_traffic(TRAFFIC_SUMMARY) if tname == "hahn_inv_cols" else None
    traffic = rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"] if rec else None
    out = {
        "metric": "CJT coefficients/sec (fwd+inv) batched N=2^16; p99 latency; rel. error",
        "value": coeffs_per_step / t_step,
        "unit": "coefficients/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"batch of {count} forward+inverse CJTs at N={N}, (alpha,beta)~U(-1/2,1/2)^2, "
                               f"c_n=randn/(n+1)", "count": count, "N": N, "seed": args.seed,
                   "parallelism": "single GPU"},
        "p50_ms": float(np.percentile(r64["per"], 50)),
        "p99_ms": float(np.percentile(r64["per"], 99)),
        "rel_error": err,
        "plan_s": {"fp64": t_plan64, "fp32_bulk": t_plan32},
        "autotune": tuned,
        "kernels_ms_per_step": {k: v["total_ms"] / args.steps for k, v in kern.items()},
        "roofline": {"bound": "alu" if alu_bound else "hbm", "kernel": tname, "achieved": achieved,
                     "peak": ceiling, "unit": unit, "frac": achieved / ceiling, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "launches_per_step": launches / args.steps, "launch_ms": t_launch * 1e3,
                     "alg_bytes_per_launch": alg_bytes, "alg_flops_per_launch": alg_flops,
                     "hbm_GBps_alg": alg_bytes / t_launch / 1e9,
                     "hbm_GBps_measured": traffic / t_launch / 1e9 if traffic else None},
        "cpu_baseline": cpu,
        "workloads": extra,
    }
    if "fp32_bulk" in results:
        r32 = results["fp32_bulk"]
        t32 = r32["wall"] / args.steps
        out["fp32_bulk"] = {"value": coeffs_per_step / t32, "ms_per_step": t32 * 1e3,
                            "p50_ms": float(np.percentile(r32["per"], 50)),
                            "p99_ms": float(np.percentile(r32["per"], 99)),
                            "speedup_vs_fp64": t_step / t32,
                            "kernels_ms_per_step": {k: v["total_ms"] / args.steps for k, v in r32["kern"].items()}}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
