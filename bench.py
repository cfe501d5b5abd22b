#!/usr/bin/env python3
"""Benchmark: Sinkhorn iterations/s of the graph-structured multi-commodity solver on one MI355X.

Default workload: the traffic-routing road grid, 100 x 100 4-neighbour roads
(n = 10^4 states with waiting self-loops), L = 2000 origin-destination
commodities, T = 120 time steps, eps = 0.05, FP32 sparse products in the
log-sum-exp domain (route costs / eps of thousands of nats).  Other workloads
(--workload): rgg2000 (random geometric graph, n = 2000, L = 256, T = 50,
scaled domain), dense4096 / dense4096_fp32 (complete graph n = 4096, L = 1024,
T = 32, BF16 or FP32 MFMA products), grid5 (5 x 5 grid, FP64), serve (the
serving trace, served vs plain).  One step = one full Sinkhorn iteration
(backward sweep, source update, forward sweep with capacity updates, sink
update); every 10th step also runs the FP64 convergence/dual check pass, as
mmot_solve does.  Inputs are resident in HBM before the timed region.  The line
also carries the serving half of the metric, measured after the timed region on
a bounded trace (48 requests at 1.5x the plain solver's capacity): served vs
plain p50/p99 latency and solves/s.

Prints one JSON line (see the "roofline" and "cpu_baseline" fields).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Sinkhorn iters/s + % HBM/MFMA roofline; p50/p99 solve latency, served vs plain"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE
# passes scaled by the counters' reading for a plain 256 MiB device copy (factors 2.0 and 1.0);
# the summary with its commands is in profiles/.  Reported only while the kernel source is the
# one the counters were taken from.
TRAFFIC = {
    "road100": {"source": "paper_2106_14485_amd/csrc/sweep_sparse.hip",
                "sha256": "c7ba77027e13b362439b292c6ae2aa481d6d26ebb6e63bb3f1d84c34a4d1dcaf",
                "fetch_kib": 87589.447, "write_kib": 79433.356, "fetch_scale": 2.0, "write_scale": 1.0},
    "rgg2000": {"source": "paper_2106_14485_amd/csrc/sweep_sparse.hip",
                "sha256": "c7ba77027e13b362439b292c6ae2aa481d6d26ebb6e63bb3f1d84c34a4d1dcaf",
                "fetch_kib": 2407.656, "write_kib": 2007.938, "fetch_scale": 2.0, "write_scale": 1.0},
}


def measured_traffic(name):
    import hashlib
    t = TRAFFIC.get(name)
    if t is None:
        return None
    with open(os.path.join(ROOT, t["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["sha256"]:
            return None
    return round((t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024)


def workload(name):
    from paper_2106_14485_amd import instances
    if name == "rgg2000":
        return instances.rgg_instance(n=2000, L=256, T=50, eps=0.05, seed=0), "fp32"
    if name == "road100":
        return instances.road_grid_instance(side=100, L=2000, T=120, eps=0.05, seed=0), "fp32"
    if name == "grid5":
        return instances.grid_instance(), "fp64"
    if name == "dense4096":
        return instances.dense_blob_instance(n=4096, L=1024, T=32, eps=0.02, seed=0), "bf16"
    if name == "dense4096_fp32":
        return instances.dense_blob_instance(n=4096, L=1024, T=32, eps=0.02, seed=0), "fp32"
    raise SystemExit(f"unknown workload {name}")


def _host_cpu():
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return f"host {model}, {os.cpu_count()} hardware threads"


def cpu_baseline(inst, log_domain, budget_s=20.0):
    """The FP64 oracle on the host, timed on a bounded sample of the same workload.

    Scaled-domain workloads: whole Sinkhorn iterations of the same instance, as
    many as fit the budget.  Log-domain workloads (the road grid: one oracle
    iteration over all 2000 commodities takes minutes): one log-domain
    iteration over the first Ls commodities of the same graph, T and capacities,
    with Ls sized to the budget; the oracle's time per iteration is linear in
    the commodity count (every product, update and reduction is per commodity),
    so the full-workload rate is the sample's times Ls / L."""
    from oracle import alg2
    C = inst.cost_csr()
    if not log_domain:
        p = alg2.make_problem(C, inst.eps, inst.T, inst.src, inst.dst, inst.cap, inst.state_cost)
        st = alg2.initial_state(p)
        t0 = time.perf_counter()
        alg2.iterate(p, st, 1)
        one = time.perf_counter() - t0
        k = max(1, int(budget_s / max(one, 1e-6)) - 1)
        t0 = time.perf_counter()
        alg2.iterate(p, st, k)
        dt = time.perf_counter() - t0
        return {"value": k / dt, "unit": "iters/s", "cores": 1, "kind": "oracle",
                "sample": f"{k} Sinkhorn iterations of the same instance after 1 warm-up (FP64 numpy/scipy, "
                          f"single-threaded sparse products); {_host_cpu()}"}

    def one_iter(ls):
        p = alg2.make_problem(C, inst.eps, inst.T, inst.src[:ls], inst.dst[:ls], inst.cap,
                              None if inst.state_cost is None else inst.state_cost[:ls])
        st = alg2.initial_log_state(p)
        t0 = time.perf_counter()
        alg2.iterate_log(p, st, 1)
        return time.perf_counter() - t0
    probe = 4
    t_probe = one_iter(probe)
    ls = int(min(inst.L, max(probe, probe * budget_s / max(t_probe, 1e-6))))
    dt = one_iter(ls)
    return {"value": (1.0 / dt) * ls / inst.L, "unit": "iters/s", "cores": 1, "kind": "oracle",
            "sample": f"1 log-domain Sinkhorn iteration of the same graph, T and capacities over the first "
                      f"{ls} of the {inst.L} commodities ({dt:.1f} s; the oracle's cost is linear in the "
                      f"commodity count, so the rate is scaled by {ls}/{inst.L}), after a {probe}-commodity "
                      f"sizing run (FP64 numpy/scipy log-sum-exp, single-threaded); {_host_cpu()}"}


def serving_compare(requests, load, max_iter, budget_gb, nmax, lmax, capacity=0.0, progress=0):
    """Served (continuous batching, the pool) vs plain one-at-a-time on the same
    seeded Poisson trace of the serving workload.  The plain solver's capacity is
    measured first (everything queued at t = 0) unless given; the arrival rate is
    load x that."""
    import numpy as np
    from paper_2106_14485_amd import instances as I
    from paper_2106_14485_amd.serve import latency_summary, serve, serve_plain
    reqs = I.serve_trace(num=requests, rate=1.0, seed=0, n_range=(200, nmax), L_range=(1, lmax))
    insts = [I.instance_from_request(r) for r in reqs]
    zero = np.zeros(len(insts))
    serve_plain(insts[:2], zero[:2], max_iter=max_iter)          # warm-up
    if capacity > 0:
        cap = capacity
    else:
        res0, t_plain0 = serve_plain(insts, zero, max_iter=max_iter, progress=progress)
        cap = len(insts) / t_plain0
    gaps = np.random.default_rng(1).exponential(1.0 / (load * cap), size=len(insts))
    arrivals = np.cumsum(gaps) - gaps[0]
    res_p, tp = serve_plain(insts, arrivals, max_iter=max_iter, progress=progress)
    res_s, ts = serve(insts, arrivals, budget_bytes=int(budget_gb * (1 << 30)), max_iter=max_iter,
                      progress=progress)
    sp, ss = latency_summary(res_p, tp), latency_summary(res_s, ts)
    def outcome(r):
        return (r["status"], r["stats"]["iters"] if r["status"] == 0 else None)
    iters_equal = all(outcome(a) == outcome(b) for a, b in zip(res_p, res_s))
    return {"workload": f"{len(insts)} Poisson requests (RGG or road grid, n log-uniform [200,{nmax}], "
                        f"T U{{10..120}}, L log-uniform [1,{lmax}], eps in {{0.02,0.05,0.1}}), FP32, "
                        f"tol 1e-6 or {max_iter} iterations",
            "offered_load": load, "plain_capacity_solves_per_s": cap,
            "served": ss, "plain": sp, "same_iterations_as_plain": iters_equal}


def serving(args):
    s = serving_compare(args.requests, args.load, args.max_iter, args.budget_gb, args.serve_nmax, args.serve_lmax,
                        capacity=args.plain_capacity, progress=100 if args.requests >= 200 else 0)
    out = {"metric": "p50/p99 solve latency, served vs plain", "value": s["served"]["p99_s"],
           "unit": "s (p99 latency)", "higher_is_better": False, "n_gpus": 1, "data": "synthetic",
           "config": {"workload": s["workload"], "offered_load": s["offered_load"],
                      "plain_capacity_solves_per_s": s["plain_capacity_solves_per_s"]},
           "served": s["served"], "plain": s["plain"], "same_iterations_as_plain": s["same_iterations_as_plain"]}
    print(json.dumps(out))
    return 0


def copy_probe(mib, reps=20):
    """A plain device-to-device copy of known size: the reference reading for the HBM byte
    counters (FETCH_SIZE / WRITE_SIZE per dispatch should be mib MiB each)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.rand(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "reps": reps}))
    return 0


def library_gemm(shape, reps=50):
    """Reference point for the dense products: the vendor library's plain GEMM
    (torch.matmul -> hipBLASLt) of the same shape, no epilogue, BF16 and FP32."""
    import torch
    m, k, n = (int(x) for x in shape.split(","))
    out = {"library_gemm": f"{m}x{k}x{n}", "reps": reps}
    for name, dt in (("bf16", torch.bfloat16), ("fp32", torch.float32)):
        g = torch.Generator(device="cuda").manual_seed(0)
        a = torch.randn(m, k, device="cuda", dtype=dt, generator=g)
        b = torch.randn(k, n, device="cuda", dtype=dt, generator=g)
        for _ in range(5):
            a @ b
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            a @ b
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"us": round(ms * 1e3, 2), "tflops": round(2.0 * m * k * n / ms / 1e9, 1)}
    print(json.dumps(out))
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="road100")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--requests", type=int, default=48)
    ap.add_argument("--serve-requests", type=int, default=48,
                    help="requests of the bounded serving comparison added to a solver line (0: none)")
    ap.add_argument("--serve-load", type=float, default=1.5)
    ap.add_argument("--plain-capacity", type=float, default=0.0,
                    help="solves/s of the plain solver on the trace (serve workload; measured when 0)")
    ap.add_argument("--load", type=float, default=0.8)
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--budget-gb", type=float, default=96.0)
    ap.add_argument("--serve-nmax", type=int, default=10000)
    ap.add_argument("--serve-lmax", type=int, default=512)
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="MiB: only run a plain device copy of this size (HBM counter calibration)")
    ap.add_argument("--library-gemm", default="",
                    help="M,K,N: only time the vendor library's plain GEMM of this shape (reference point)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this solver runs on one GPU; multi-GPU sharding is designed but not built "
                                   "(run with --gpus 1)"}))
        return 2

    if args.workload == "serve":
        return serving(args)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.library_gemm:
        return library_gemm(args.library_gemm)

    import torch
    from paper_2106_14485_amd.solver import Solver

    inst, prec = workload(args.workload)
    S = Solver(inst, precision=prec, domain="auto")
    check_every = 10
    # warm-up (also runs the first calibration iterations and captures the graphs)
    done = 0
    while done < args.warmup:
        k = min(check_every, args.warmup - done)
        S.iterate(k)
        done += k
    S.stats()
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        k = min(check_every, args.steps - done)
        S.iterate(k, stats=(done + k) % check_every == 0)
        done += k
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = S.stats()

    # live per-launch time of the dominant kernel (forward sweep step), HIP events
    fwd_ms = S.time_step(forward=True, reps=200)
    bwd_ms = S.time_step(forward=False, reps=200)
    n, L, T, nnz = inst.n, inst.L, inst.T, inst.nnz
    vsz = 8 if prec == "fp64" else 4
    Lp = (L + (16 // vsz) - 1) // (16 // vsz) * (16 // vsz)
    iters_per_s = args.steps / dt
    if inst.kind == "dense":
        # one forward product: OUT (n x Lp) = K^T (n x n) diag(u) B (n x Lp): 2 n^2 Lp flops
        flops = 2.0 * n * n * Lp
        achieved = flops / (fwd_ms * 1e-3) / 1e12
        peak = 2500.0 if prec == "bf16" else 157.3
        roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 5), "traffic": None, "kernel": "k_gemm_lds<false, 0> forward (BF16)" if prec == "bf16" else "k_gemm_lds<true, 0> forward (FP32)",
                "kernel_ms": round(fwd_ms, 5), "flops_per_launch": flops, "bwd_kernel_ms": round(bwd_ms, 5)}
    else:
        # algorithmic bytes of one forward step: read hatPsi_t, read Psi_{t+1}, write hatPsi_{t+1}
        # (3 panels of n x Lp) + operator (8 B per CSR entry) + u_t, u_{t+1}, d (3 x 4 B per state)
        fwd_bytes = 3 * n * Lp * vsz + nnz * (4 + vsz) + 3 * n * vsz + (n + 1) * 4
        achieved = fwd_bytes / (fwd_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(args.workload),
                "kernel": "k_ell_step forward (capacity epilogue)", "kernel_ms": round(fwd_ms, 5),
                "bytes_per_launch": fwd_bytes, "bwd_kernel_ms": round(bwd_ms, 5)}
    out = {
        "metric": METRIC,
        "value": round(iters_per_s, 3),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{inst.name}: n={n} states (nnz={nnz}), L={L} commodities, T={T}, "
                               f"eps={inst.eps}, {prec.upper()} {inst.kind.upper()}, "
                               f"domain={'log' if st['domain'] == 2 else 'scaled'}",
                   "check_every": check_every, "keep_forward": int(S.opts.keep_forward)},
        "roofline": roof,
        "stats": {k: st[k] for k in ("dual_obj", "src_resid", "cap_viol", "mass_drift")},
    }
    S.close()
    del S
    if not args.no_cpu_baseline and inst.kind == "csr":
        out["cpu_baseline"] = cpu_baseline(inst, st["domain"] == 2, args.cpu_budget)
    if args.serve_requests > 0:
        # the serving half of the metric on a bounded trace: served vs plain p50/p99 and solves/s
        out["serving"] = serving_compare(args.serve_requests, args.serve_load, args.max_iter, args.budget_gb,
                                         args.serve_nmax, args.serve_lmax)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
