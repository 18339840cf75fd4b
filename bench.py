"""Throughput of the adaptive FP64 solve on one MI355X.

One step solves the five single large systems of the paper-shaped workload
once each (dense general n=8192, SPD n=8192, lower-triangular n=8192 with
scaled off-diagonals, banded n=1,000,000 with kl=ku=5 in band layout, and
symmetric-indefinite n=4096, whose Cholesky fails and re-routes to LU), with
nrhs right-hand sides each. Inputs are seeded, synthetic and resident in HBM
before the timed region; every solve's backward error is checked against the
1e-10 bar. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--nrhs 1|64] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2007_11208_amd import workloads as W  # noqa: E402

METRIC = "solves/s + TFLOP/s vs plain FP64 solve at ≤1e-10 backward err; p50/p99 latency"
SYSTEMS = ("dense", "spd", "lower_scaled", "banded", "symindef")
BERR_BAR = 1e-10

# single-kernel families and the kernel behind each (the roofline is quoted for one kernel)
FAMILY_KERNEL = {
    "gemm": ("k_gemm_sub", "gemm.hip", "mfma"),
    "panel": ("k_getrf_panel", "lu.hip", "hbm"),
    "laswp": ("k_laswp_moves", "lu.hip", "hbm"),
    "trsm_block": ("k_trsm_lines", "trsm_lines.hip", "alu"),
    "potrf": ("k_potrf_diag", "chol.hip", "alu"),
    "trsv": ("k_trsv1", "trsv.hip", "hbm"),
    "gbtrf": ("k_gbtrf_k", "band.hip", "hbm"),
    "detect": ("k_detect_dense", "detect.hip", "hbm"),
}
PEAK = {"mfma": (78.6, "TFLOP/s"), "alu": (78.6, "TFLOP/s"), "hbm": (8000.0, "GB/s"), "mfma32": (157.3, "TFLOP/s"),
        "mfma16": (2500.0, "TFLOP/s")}


def algorithmic_flops(name: str, n: int, nrhs: int, route: str, kl: int = 0, ku: int = 0) -> float:
    """Flops the routed method must do (factorisation + solve), not the dense work it avoids."""
    if route == "lu":
        return 2.0 * n ** 3 / 3.0 + 2.0 * n * n * nrhs
    if route == "chol":
        return n ** 3 / 3.0 + 2.0 * n * n * nrhs
    if route == "tri":
        return float(n) * n * nrhs
    if route == "band_lu":
        return 2.0 * n * kl * (kl + ku) + 2.0 * n * (2 * kl + ku + 1) * nrhs
    return float("nan")


def pct(v, q):
    return float(np.percentile(np.asarray(v), q)) if len(v) else float("nan")


def traffic_for(kernel_src: str, kernel: str):
    """Measured HBM bytes per launch from the committed counter summary, if the kernel is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    ent = table.get(kernel)
    if not ent:
        return None
    with open(os.path.join(ROOT, "paper_2007_11208_amd", "csrc", kernel_src), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if ent.get("src_sha256") != sha:
        return None
    return ent.get("bytes_per_launch")


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(host_cases):
    """The oracle on this host's cores, at full size, on the same inputs the GPU solved: one oracle
    solve of each system with every core; the two systems whose oracle solve is O(n^2) or less
    (banded, lower triangular) also on one thread."""
    import oracle
    O = oracle.get()
    cores = O.num_threads()

    def one(name, a, b, lay):
        t0 = time.perf_counter()
        if lay[0] == "band":
            O.solve_band(a, lay[1], lay[2], b)
        else:
            O.solve(a, b)
        return time.perf_counter() - t0

    per = {name: one(name, a, b, lay) for name, a, b, lay in host_cases}
    single = {}
    O.set_threads(1)
    try:
        for name, a, b, lay in host_cases:
            if name in ("banded", "lower_scaled"):
                single[name] = round(one(name, a, b, lay), 4)
    finally:
        O.set_threads(cores)
    step = sum(per.values())
    return {"value": len(per) / step, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": "one oracle solve of each system of the step at full size, on the same inputs as the GPU",
            "per_system_s": {k: round(v, 4) for k, v in per.items()}, "single_thread_s": single,
            "cpu_model": host_cpu_model(), "host_cpus": os.cpu_count()}


def oracle_backward_errors(host_cases, xs):
    """The oracle's backward error of each x the GPU returned (exact products, compensated sums)."""
    import oracle
    O = oracle.get()
    out = {}
    for (name, a, b, lay), x in zip(host_cases, xs):
        if lay[0] == "band":
            out[name] = float(O.berr_band(a, lay[1], lay[2], b, x))
        else:
            out[name] = float(O.berr(a, b, x)[0])
    return out


def batched_flops(kind_route, n, nrhs):
    route = kind_route
    if route in ("lu", "band_lu"):
        return 2.0 * n ** 3 / 3.0 + 2.0 * n * n * nrhs
    if route == "chol":
        return n ** 3 / 3.0 + 2.0 * n * n * nrhs
    if route == "tri":
        return float(n) * n * nrhs
    return 0.0  # the SVD route: not counted as useful work


def bench_batched(args):
    """Many small systems (sizes, class mix and right-hand sides of the batched configuration)
    solved by one ada_solve_batched launch per step."""
    import torch
    from paper_2007_11208_amd import ada
    n_lo, n_hi = (int(v) for v in args.n_range.split(","))
    cases = W.batched_case(args.count, k=0, n_lo=n_lo, n_hi=n_hi)
    As = [c[1] for c in cases]
    Bs = [c[2] for c in cases]
    batch = ada.Batch(As, Bs, precision=args.precision)
    for _ in range(args.warmup):
        batch.run()
    torch.cuda.synchronize()
    # the launch shape: the autotuner's choice for this batch (set-up, outside the timed region)
    tuned = None
    if not args.no_tune:
        t_tune = time.perf_counter()
        shape, tuned_ms = batch.tune()
        torch.cuda.synchronize()
        tuned = {"shape": shape, "ms_per_batch": round(tuned_ms, 3), "tune_s": round(time.perf_counter() - t_tune, 2)}
    times = []
    ev = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()  # the batch runs on torch's current stream
        batch.run()
        e1.record()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - s0)
        ev.append(e0.elapsed_time(e1) * 1e-3)
    total = time.perf_counter() - t0
    res = batch.results()
    worst = max((r.berr for r in res), default=0.0)
    bad = [k for k, r in enumerate(res) if r.status != 0 or not (r.berr <= BERR_BAR)]
    if bad:
        print(f"{len(bad)} systems failed or missed the backward-error bar (first {bad[:5]})", file=sys.stderr)
        sys.exit(1)
    flops = sum(batched_flops(r.route, a.shape[0], b.shape[1]) for r, a, b in zip(res, As, Bs))
    routes = {}
    for r in res:
        routes[r.route] = routes.get(r.route, 0) + 1
    refine = None
    if args.precision == "fp32_ir":
        its = [r.refine_iters for r in res if r.route in ("lu", "chol", "band_lu") or r.refine_iters < 0]
        conv = [i for i in its if i > 0]
        refine = {"refined": len(conv), "to_fp64": sum(1 for i in its if i < 0),
                  "iters_mean": round(float(np.mean(conv)), 3) if conv else None,
                  "iters_max": max(conv) if conv else None}
    value = args.count * args.steps / total
    kern_s = float(np.mean(ev))
    achieved = flops / kern_s / 1e12
    roof = {"bound": "alu", "achieved": round(achieved, 4), "peak": 78.6, "unit": "TFLOP/s",
            "frac": round(achieved / 78.6, 5), "traffic": None, "kernel": "k_solve_batched",
            "avg_launch_ms": round(kern_s * 1e3, 3)}
    cpu = None
    if not args.no_cpu:
        import oracle
        O = oracle.get()
        t = time.perf_counter()
        m = 0
        for a, b in zip(As, Bs):
            O.solve(a, b)
            m += 1
            if time.perf_counter() - t > 20.0:
                break
        dt = time.perf_counter() - t
        cpu = {"value": m / dt, "unit": "solves/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"the first {m} systems of the same batch, one oracle solve each"}
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"batched ({args.precision}): {args.count} systems, n uniform in [{n_lo}, {n_hi}], nrhs uniform in [1, 8], "
                               "40% dense general, 30% SPD, 15% banded, 10% triangular, 5% condition 1e15",
                   "count": args.count},
        "tflops": round(flops * args.steps / total / 1e12, 4),
        "p50_step_ms": round(pct(times, 50) * 1e3, 3), "p99_step_ms": round(pct(times, 99) * 1e3, 3),
        "max_berr": worst, "routes": routes, "refinement": refine, "launch_shape": batch.shape(), "autotune": tuned,
        "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def spectrum_system_gpu(n, kappa, spd, nrhs, seed, dev):
    """The prescribed-spectrum system of the mixed-precision configuration, generated on the device
    (input generation, outside the timed solves)."""
    a, b, _ = W.spectrum_system_torch(n, kappa, spd, nrhs, seed, dev)
    return a, b


def bench_mixed(args):
    """Mixed precision against plain FP64 on the same systems: dense and SPD with a prescribed
    spectrum, nrhs right-hand sides, each solved in FP64, with FP32 and with BF16 trailing updates
    (FP64 refinement). Reports refinement steps, final backward error and time per solve."""
    import torch
    from paper_2007_11208_amd import ada
    dev = torch.device("cuda:0")
    sizes = [int(v) for v in args.mixed_n.split(",") if v]
    kappas = [float(v) for v in args.mixed_kappa.split(",") if v]
    precs = ("fp64", "fp32_ir", "bf16_ir")
    ctx = ada.context(0)
    rows = []
    tot = {p: 0.0 for p in precs}
    flops = 0.0
    worst = {p: 0.0 for p in precs}
    k = 0
    for kind in ("dense", "spd"):
        for n in sizes:
            for kappa in kappas:
                A, B = spectrum_system_gpu(n, kappa, kind == "spd", args.nrhs, 200 + k, dev)
                k += 1
                X = torch.empty((args.nrhs, n), dtype=torch.float64, device=dev).t()
                opts = ada.make_opts()
                work = torch.empty(ada.workspace_size(n, args.nrhs, opts), dtype=torch.uint8, device=dev)
                torch.cuda.synchronize()
                row = {"kind": kind, "n": n, "kappa": kappa}
                for p in precs:
                    for _ in range(args.warmup):
                        ada.solve(A, B, out=X, work=work, ctx=ctx, precision=p)
                    ts = []
                    for _ in range(args.steps):
                        t0 = time.perf_counter()
                        _, r = ada.solve(A, B, out=X, work=work, ctx=ctx, precision=p)
                        ts.append(time.perf_counter() - t0)
                    t = float(np.median(ts))
                    tot[p] += t
                    worst[p] = max(worst[p], r.berr)
                    row[p] = {"ms": round(t * 1e3, 3), "route": r.route, "refine_iters": r.refine_iters,
                              "berr": r.berr, "rcond": r.rcond}
                    if not (r.berr <= BERR_BAR):
                        print(f"{kind} n={n} kappa={kappa} {p}: backward error {r.berr} above {BERR_BAR}",
                              file=sys.stderr)
                        sys.exit(1)
                flops += (2.0 if kind == "dense" else 1.0) * n ** 3 / 3.0 + 2.0 * n * n * args.nrhs
                print(json.dumps({"case": row}), flush=True)
                rows.append(row)
                del A, B, X, work
                torch.cuda.empty_cache()
    # achieved rate of the low-precision trailing update (FP32 operands) on the largest dense case
    n = sizes[-1]
    A, B = spectrum_system_gpu(n, kappas[0], False, args.nrhs, 999, dev)
    X = torch.empty((args.nrhs, n), dtype=torch.float64, device=dev).t()
    work = torch.empty(ada.workspace_size(n, args.nrhs, ada.make_opts()), dtype=torch.uint8, device=dev)
    ada.solve(A, B, out=X, work=work, ctx=ctx, precision="fp32_ir")
    ctx.profile_reset()
    ctx.profile(True)
    ada.solve(A, B, out=X, work=work, ctx=ctx, precision="fp32_ir")
    ctx.profile(False)
    launches, ms, fl, by = ctx.profile_read("gemm")
    achieved = fl / (ms * 1e-3) / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK["mfma32"][0], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK["mfma32"][0], 5), "traffic": None, "kernel": "k_gemm_sub_f32",
            "launches": launches, "avg_us": round(ms * 1e3 / max(1, launches), 2)}
    nsys = len(rows)
    out = {
        "metric": METRIC, "value": round(nsys / tot["fp32_ir"], 4), "unit": "solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(tot["fp32_ir"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"mixed precision: dense and SPD U diag(s) V^T, n in {sizes}, kappa in {kappas}, "
                               f"nrhs={args.nrhs}; one step = every system once (median of {args.steps} solves each)"},
        "solves_per_s": {p: round(nsys / tot[p], 4) for p in precs},
        "tflops": {p: round(flops / tot[p] / 1e12, 4) for p in precs},
        "speedup_vs_fp64": {p: round(tot["fp64"] / tot[p], 3) for p in precs},
        "max_berr": worst, "roofline": roof, "cpu_baseline": None, "cases": rows,
    }
    print(json.dumps(out), flush=True)


def bench_paper(args):
    """The paper's own comparisons on the GPU (Section III, Tables I-IV): each system solved one call at a
    time through ada_solve, timed per call with events on the solve's stream (device) and on the host
    clock around call + synchronize (wall).

    * small: the five seeded systems of the small configuration (dense, SPD, upper-triangular n=256,
      banded n=1024 kl=ku=2, ill-conditioned n=64 that must take the SVD fallback), --paper-reps calls each;
    * compare: adaptive against the plain LU route (force_general: LU with partial pivoting, its solve and
      the condition estimate, the 'standard' solver of Section II-D) on banded (kl=ku=2, five diagonals),
      lower-triangular (off-diagonals scaled by 1/sqrt(n), so that the triangular route is the one taken),
      SPD and dense systems at n in {100, 250, 500, 1000}: a pool of eight seeded systems per cell,
      --paper-reps calls cycling through it, p50/p99 per call and the speedup of the medians;
    * lower_literal: the lower-triangular n=8192 system with N(0,1) off-diagonals as the large
      configuration states it; its condition number grows exponentially with n, so the rule of Section
      II-E sends it to the SVD fallback (one call, --no-literal skips it)."""
    import torch
    from paper_2007_11208_amd import ada
    dev = torch.device("cuda:0")
    ctx = ada.context(0)
    stream = torch.cuda.current_stream(dev)
    reps = args.paper_reps

    def timed_calls(systems, k_calls, **kw):
        dev_ms, wall_ms, res = [], [], []
        work = None
        outs = [torch.empty((b.shape[1], b.shape[0]), dtype=torch.float64, device=dev).t() for _, b in systems]
        for (A, B), X in zip(systems, outs):  # warm-up: one call per system
            ada.solve(A, B, out=X, ctx=ctx, **kw)
        torch.cuda.synchronize()
        for k in range(k_calls):
            A, B = systems[k % len(systems)]
            X = outs[k % len(systems)]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0 = time.perf_counter()
            e0.record(stream)
            _, r = ada.solve(A, B, out=X, ctx=ctx, **kw)
            e1.record(stream)
            torch.cuda.synchronize()
            wall_ms.append((time.perf_counter() - t0) * 1e3)
            dev_ms.append(e0.elapsed_time(e1))
            if k < len(systems):
                res.append(r)
        return dev_ms, wall_ms, res

    def stats(v):
        return {"p50": round(pct(v, 50), 4), "p99": round(pct(v, 99), 4), "mean": round(float(np.mean(v)), 4)}

    to_dev = lambda a: torch.from_numpy(np.asfortranarray(a)).to(dev)
    out = {"metric": METRIC, "workload": "paper", "n_gpus": 1, "data": "synthetic", "dtype": "f64", "reps": reps}
    # small configuration
    small = {}
    for name in ("a_dense", "b_spd", "c_upper", "d_banded", "e_illcond"):
        a, b = W.small_case(name)
        sysd = [(to_dev(a), to_dev(b))]
        dms, wms, res = timed_calls(sysd, reps)
        r = res[0]
        if r.status == 0 and not (r.berr <= BERR_BAR):
            print(f"{name}: backward error {r.berr} above the bar", file=sys.stderr)
            sys.exit(1)
        small[name] = {"n": a.shape[0], "class": r.cls, "route": r.route, "rcond": r.rcond, "rank": r.rank,
                       "berr": r.berr, "device_ms": stats(dms), "wall_ms": stats(wms)}
        print(f"small {name}: {r.cls}/{r.route} device p50 {pct(dms, 50):.3f} ms p99 {pct(dms, 99):.3f} ms",
              file=sys.stderr, flush=True)
    out["small"] = small
    # adaptive against the plain LU route
    gens = {"banded": lambda n, g: W.banded_dense(n, 2, 2, g),
            "lower_triangular": lambda n, g: W.triangular(n, g, upper=False, scaled=True),
            "spd": W.spd, "dense": W.dense_general}
    comp = []
    for cname, gen in gens.items():
        for n in (100, 250, 500, 1000):
            g = np.random.default_rng(7000 + n)
            pool = []
            for _ in range(8):
                a = gen(n, g)
                x = W.x_true(n, 1, g)
                pool.append((to_dev(a), to_dev(W.rhs_for(a, x))))
            ad, aw, ar = timed_calls(pool, reps)
            gd, gw, gr = timed_calls(pool, reps, force_general=True)
            worst = max(r.berr for r in ar + gr)
            if not (worst <= BERR_BAR):
                print(f"{cname} n={n}: backward error {worst} above the bar", file=sys.stderr)
                sys.exit(1)
            row = {"class": cname, "n": n, "route": ar[0].route, "general_route": gr[0].route,
                   "adaptive_device_ms": stats(ad), "general_device_ms": stats(gd),
                   "adaptive_wall_ms": stats(aw), "general_wall_ms": stats(gw),
                   "speedup_p50_device": round(pct(gd, 50) / pct(ad, 50), 3),
                   "speedup_p50_wall": round(pct(gw, 50) / pct(aw, 50), 3)}
            comp.append(row)
            print(f"compare {cname} n={n}: {row['route']} {pct(ad, 50):.3f} ms vs lu {pct(gd, 50):.3f} ms "
                  f"-> x{row['speedup_p50_device']}", file=sys.stderr, flush=True)
    out["compare"] = comp
    # the literal lower-triangular system of the large configuration
    if not args.no_literal:
        a, b, _ = W.large_case("lower")
        A, B = to_dev(a), to_dev(b)
        del a
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, r = ada.solve(A, B, ctx=ctx)
        e1.record(stream)
        torch.cuda.synchronize()
        out["lower_literal"] = {"n": 8192, "class": r.cls, "route": r.route, "fallback": r.fallback,
                                "rcond": r.rcond, "rank": r.rank, "sweeps": r.sweeps, "berr": r.berr,
                                "status": r.status, "device_ms": round(e0.elapsed_time(e1), 3),
                                "wall_ms": round((time.perf_counter() - t0) * 1e3, 3)}
        print(f"lower_literal: {r.cls}/{r.route} rcond {r.rcond:.3e} rank {r.rank} sweeps {r.sweeps} "
              f"{out['lower_literal']['device_ms']:.1f} ms", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def bench_serving(args):
    """Poisson request stream into the solve server: requests draw a system from a seeded pool
    (sizes log-uniform in [16, 4096], the batched class mix); a fraction reuse one of the
    resident factorisations with a new right-hand side. Latency is submission to completion as
    the server records it; throughput is completed requests over the span from the first
    submission to the last completion."""
    import threading
    import torch
    from paper_2007_11208_amd import ada
    dev = torch.device("cuda:0")
    pool = [W.serving_system(k) for k in range(args.pool)]
    dA = [torch.from_numpy(np.asfortranarray(a)).to(dev) for _, a, _ in pool]
    dB = [torch.from_numpy(np.asfortranarray(b)).to(dev) for _, _, b in pool]
    free, total = torch.cuda.mem_get_info(dev)
    arena = int(min(args.arena_gb * (1 << 30), free - (8 << 30)))
    srv = ada.Server(arena, solve_workers=args.workers)
    # resident factors: the first systems of the pool, kept before the stream starts
    resident = []
    for k in range(min(args.resident, len(pool))):
        rc, r, _, f, _, _ = srv.poll(srv.submit(dA[k], dB[k], keep=True))
        if rc != 0:
            print(f"keeping factors of pool system {k} failed: {rc} {ada.last_error()}", file=sys.stderr)
            sys.exit(1)
        g = torch.Generator(device=dev)
        g.manual_seed(500 + k)
        bn = torch.randn(dB[k].shape[1], dB[k].shape[0], dtype=torch.float64, device=dev, generator=g).t()
        resident.append((k, f, bn))
    arrivals = W.poisson_arrivals(args.rate, args.duration, seed=4)
    g = np.random.default_rng(44)
    reuse = g.random(len(arrivals)) < args.reuse
    pick_pool = g.integers(0, len(pool), len(arrivals))
    pick_res = g.integers(0, max(1, len(resident)), len(arrivals))
    tickets = []
    meta = []
    lock = threading.Lock()
    done = []
    sub_done = threading.Event()

    def drain():
        i = 0
        while True:
            with lock:
                have = i < len(tickets)
                t = tickets[i] if have else None
            if not have:
                if sub_done.is_set():
                    with lock:
                        if i >= len(tickets):
                            return
                    continue
                time.sleep(0.0005)
                continue
            out = srv.poll(t, timeout_us=100000)
            if out is None:
                if time.perf_counter() - t0 > args.max_wait:
                    return  # stop waiting: the rest is reported as unfinished
                continue
            done.append((i, out[0], out[1], out[4], out[5], time.perf_counter()))
            i += 1
            if i % 1000 == 0:
                print(f"served {i} of {len(arrivals)} at {time.perf_counter() - t0:.1f} s", file=sys.stderr,
                      flush=True)

    th = threading.Thread(target=drain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    th.start()
    late = 0.0
    for i, ta in enumerate(arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        else:
            late = max(late, now - ta)
        if reuse[i] and resident:
            k, f, bn = resident[pick_res[i]]
            t = srv.submit(None, bn, reuse=f)
            kind = "reuse"
            n = dA[k].shape[0]
        else:
            k = int(pick_pool[i])
            t = srv.submit(dA[k], dB[k])
            n = dA[k].shape[0]
            kind = "batched" if n <= 256 and dB[k].shape[1] <= 8 else "single"
        with lock:
            tickets.append(t)
            meta.append((kind, n, pool[k][0]))
    sub_done.set()
    th.join()
    if not done:
        print("no request completed", file=sys.stderr)
        sys.exit(1)
    t_end = max(d[5] for d in done)
    span = t_end - t0
    lat = np.array([d[4] for d in done]) * 1e-3  # ms
    statuses = {}
    worst = 0.0
    by_kind = {}
    by_class = {}
    for (i, rc, r, q_us, tot_us, _) in done:
        statuses[rc] = statuses.get(rc, 0) + 1
        if rc == 0 and r.berr == r.berr:
            worst = max(worst, r.berr)
        kind, n, cls = meta[i]
        by_kind.setdefault(kind, []).append(tot_us * 1e-3)
        by_class.setdefault(r.route, []).append(tot_us * 1e-3)
    ok_bar = sum(1 for (i, rc, r, _, _, _) in done if rc == 0 and r.berr <= BERR_BAR)

    def summ(v):
        return {"count": len(v), "p50_ms": round(pct(v, 50), 3), "p99_ms": round(pct(v, 99), 3)}

    unfinished = len(arrivals) - len(done)
    srv.close()  # drops what never started; waits for what runs
    out = {
        "metric": METRIC, "value": round(len(done) / span, 2), "unit": "solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(span * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:g} req/s for {args.duration:g} s, n log-uniform in "
                               f"[16, 4096] (pool of {len(pool)} seeded systems), 40% dense / 30% SPD / 15% banded / "
                               f"10% triangular / 5% condition 1e15, {args.reuse:.0%} reuse of {len(resident)} resident "
                               f"factorisations, arena {arena / (1 << 30):.1f} GiB, {args.workers} solve workers"},
        "offered_rate": args.rate, "requests": len(done), "unfinished": unfinished, "p50_ms": round(float(np.median(lat)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3), "by_kind": {k: summ(v) for k, v in by_kind.items()},
        "by_route": {k: summ(v) for k, v in by_class.items()}, "status_counts": statuses,
        "met_berr_bar": ok_bar, "max_berr": worst, "submit_lag_ms": round(late * 1e3, 3),
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(out), flush=True)


def bench_extensions(args, cases, ctx, dev):
    """The routes the paper names as future work, beside the paper's routes on the same systems:
    the symmetric-indefinite system (Cholesky fails; LU vs LDL^T) and a plain symmetric n=4096 system
    (LU vs LDL^T)."""
    import torch
    from paper_2007_11208_amd import ada
    out = {}

    def timed(label, A, B, X, work, exts, **kw):
        ts, r = [], None
        ctx.profile_reset()
        for k in range(args.ext_steps + 1):
            if k == 1:
                ctx.profile(True)
            t0 = time.perf_counter()
            _, r = ada.solve(A, B, out=X, work=work, ctx=ctx, extensions=exts, **kw)
            if k:
                ts.append(time.perf_counter() - t0)
        ctx.profile(False)
        pr = ctx.profile_all()
        if not (r.berr <= BERR_BAR):
            print(f"backward error {r.berr} of {label} above {BERR_BAR}", file=sys.stderr)
            sys.exit(1)
        pl = pr["panel"]
        out[label] = {"route": r.route, "chol_failed": r.chol_failed, "berr": r.berr, "rcond": r.rcond,
                      "p50_ms": round(pct(ts, 50) * 1e3, 3),
                      "panel_avg_us": round(pl[1] * 1e3 / pl[0], 2) if pl[0] else None,
                      "panel_ms_per_solve": round(pl[1] / len(ts), 3)}

    sym = [c for c in cases if c[0] == "symindef"]
    if sym:
        name, A, B, kw, work, X, n = sym[0]
        for label, exts in (("symindef_paper", ()), ("symindef_ldlt", ("sym",))):
            timed(label, A, B, X, work, exts)
        g = torch.Generator(device=dev).manual_seed(4242)
        M = torch.randn((n, n), generator=g, dtype=torch.float64, device=dev)
        M = (M + M.t()).contiguous().t()  # column-major storage of the symmetric matrix
        for label, exts in (("plain_sym_n4096_paper", ()), ("plain_sym_n4096_ldlt", ("sym",))):
            timed(label, M, B, X, work, exts)
        del M
    torch.cuda.synchronize()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nrhs", type=int, default=None, help="right-hand sides (default 1; 16 for --workload mixed)")
    ap.add_argument("--systems", default=",".join(SYSTEMS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="single", choices=("single", "batched", "mixed", "serving", "paper"),
                    help="single: the five large systems; batched: many small systems in one launch per step")
    ap.add_argument("--count", type=int, default=20000, help="systems per step of the batched workload")
    ap.add_argument("--n-range", default="8,256", help="batched workload: smallest and largest order")
    ap.add_argument("--no-tune", action="store_true", help="batched workload: keep the default launch shape")
    ap.add_argument("--paper-reps", type=int, default=1000, help="paper workload: timed calls per system or cell")
    ap.add_argument("--no-literal", action="store_true",
                    help="paper workload: skip the literal lower-triangular n=8192 system (SVD fallback)")
    ap.add_argument("--ext-steps", type=int, default=3,
                    help="single workload: also time the Section V extension route (LDL^T) "
                         "against the paper's routes on systems of the same shapes")
    ap.add_argument("--concurrent-steps", type=int, default=3,
                    help="single workload: also time this many steps with the systems solved concurrently "
                         "(one stream each; reported beside the sequential value); 0: skip")
    ap.add_argument("--mixed-n", default="4096,8192,16384", help="mixed workload: orders")
    ap.add_argument("--rate", type=float, default=2000.0, help="serving: offered requests per second")
    ap.add_argument("--duration", type=float, default=1.0, help="serving: seconds of arrivals")
    ap.add_argument("--max-wait", type=float, default=120.0,
                    help="serving: stop waiting for completions this many seconds after the first arrival")
    ap.add_argument("--pool", type=int, default=64, help="serving: distinct seeded systems")
    ap.add_argument("--resident", type=int, default=16, help="serving: resident factorisations")
    ap.add_argument("--reuse", type=float, default=0.3, help="serving: fraction of requests that reuse one")
    ap.add_argument("--workers", type=int, default=3, help="serving: solve workers")
    ap.add_argument("--arena-gb", type=float, default=200.0, help="serving: admission cap (GiB)")
    ap.add_argument("--mixed-kappa", default="1e2,1e5,1e8", help="mixed workload: condition numbers")
    ap.add_argument("--precision", default="fp64", choices=("fp64", "fp32_ir"),
                    help="batched workload: FP64 factors, or FP32 factors with FP64 iterative refinement")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only copy this many MiB device-to-device three times (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.nrhs is None:
        args.nrhs = 16 if args.workload == "mixed" else 1
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs each system on a single device; "
              "run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2007_11208_amd import ada

    dev = torch.device("cuda:0")
    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib * (1 << 20) // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return
    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "mixed":
        return bench_mixed(args)
    if args.workload == "serving":
        return bench_serving(args)
    if args.workload == "paper":
        return bench_paper(args)
    names = [s for s in args.systems.split(",") if s]
    cases = []
    host_cases = []  # the same inputs on the host, for the oracle after the timed region
    for name in names:
        a, b, lay = W.large_case(name, nrhs=args.nrhs)
        host_cases.append((name, a, b, lay))
        A = torch.from_numpy(np.asfortranarray(a)).to(dev)
        B = torch.from_numpy(np.asfortranarray(b)).to(dev)
        kw = dict(layout="band", kl_in=lay[1], ku_in=lay[2]) if lay[0] == "band" else {}
        n = B.shape[0]
        opts = ada.make_opts(layout=ada.LAYOUT_BAND if kw else ada.LAYOUT_DENSE, kl_in=kw.get("kl_in", 0),
                             ku_in=kw.get("ku_in", 0))
        work = torch.empty(ada.workspace_size(n, args.nrhs, opts), dtype=torch.uint8, device=dev)
        X = torch.empty((args.nrhs, n), dtype=torch.float64, device=dev).t()
        cases.append((name, A, B, kw, work, X, n))
    torch.cuda.synchronize()
    ctx = ada.context(0)
    # set-up, not timed: the band-solve autotuner picks its LDS staging piece for the band widths
    tuned = {}
    for name, A, B, kw, work, X, n in cases:
        if kw and kw["kl_in"] + kw["ku_in"] >= 1:
            tuned[name] = ctx.autotune_band(n, kw["kl_in"], kw["ku_in"], args.nrhs)[0]

    def step(lat, info):
        for name, A, B, kw, work, X, n in cases:
            t0 = time.perf_counter()
            _, r = ada.solve(A, B, out=X, work=work, ctx=ctx, **kw)  # returns after the result is known
            dt = time.perf_counter() - t0
            if lat is not None:
                lat[name].append(dt)
                info[name] = r

    for _ in range(args.warmup):
        step(None, None)
    # one more untimed step with every kernel family timed: the per-family breakdown and the dominant
    # family; the timed steps then bracket only that family's launches with events (an event is a
    # packet between dependent kernels, and timing every launch slows the step by about 5%)
    ctx.profile_reset()
    ctx.profile(True)
    step(None, None)
    torch.cuda.synchronize()
    ctx.profile(False)
    prof_all = ctx.profile_all()
    fam = max(FAMILY_KERNEL, key=lambda f: prof_all[f][1])
    lat = {c[0]: [] for c in cases}
    info = {}
    ctx.profile_reset()
    ctx.profile(True, families=[fam])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_times = []
    for _ in range(args.steps):
        s0 = time.perf_counter()
        step(lat, info)
        step_times.append(time.perf_counter() - s0)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ctx.profile(False)
    prof = ctx.profile_all()

    per_sys = {}
    flops_step = 0.0
    worst_berr = 0.0
    for name, A, B, kw, work, X, n in cases:
        r = info[name]
        fl = algorithmic_flops(name, n, args.nrhs, r.route, r.kl, r.ku)
        flops_step += fl
        worst_berr = max(worst_berr, r.berr)
        per_sys[name] = {"n": n, "class": r.cls, "route": r.route, "rcond": r.rcond, "berr": r.berr,
                         **({"band_piece": tuned[name]} if name in tuned else {}),
                         "p50_ms": round(pct(lat[name], 50) * 1e3, 3), "p99_ms": round(pct(lat[name], 99) * 1e3, 3),
                         "tflops": round(fl / pct(lat[name], 50) / 1e12, 4)}
        if not (r.berr <= BERR_BAR):
            print(f"backward error {r.berr} of {name} above {BERR_BAR}", file=sys.stderr)
            sys.exit(1)

    nsolves = len(cases) * args.steps
    value = nsolves / total

    # after the timed region: the oracle's backward error of every x the GPU returned, which the
    # library's own value must match
    xs_host = [np.asfortranarray(c[5].cpu().numpy()) for c in cases]
    oracle_eta = oracle_backward_errors(host_cases, xs_host)
    for name, _, _, _, _, _, _ in cases:
        eo, eg = oracle_eta[name], info[name].berr
        per_sys[name]["berr_oracle"] = eo
        if not (eo <= BERR_BAR) or not (abs(eg - eo) <= 1e-6 * eo + 1e-300):
            print(f"{name}: oracle backward error {eo} (library {eg}) misses the bar or disagrees",
                  file=sys.stderr)
            sys.exit(1)

    # roofline of the dominant single-kernel family over the timed region
    launches, ms, fl, by = prof[fam]
    kernel, src, bound = FAMILY_KERNEL[fam]
    peak, unit = PEAK[bound]
    if bound == "hbm":
        achieved = by / (ms * 1e-3) / 1e9
    else:
        achieved = fl / (ms * 1e-3) / 1e12
    traffic = traffic_for(src, kernel)
    roofline = {"bound": bound, "achieved": round(achieved, 4), "peak": peak, "unit": unit,
                "frac": round(achieved / peak, 6), "traffic": traffic, "kernel": kernel,
                "launches": launches, "avg_us": round(ms * 1e3 / max(1, launches), 2),
                "share_of_step": round(ms * 1e-3 / total, 4),
                "per_launch": {"flops": fl / max(1, launches), "bytes": by / max(1, launches)}}
    families = {f: {"launches": v[0], "ms": round(v[1], 3)} for f, v in prof_all.items() if v[0]}

    # the same systems solved concurrently: one host thread, context and HIP stream each, so that the
    # latency-bound chains of different systems share the device (reported beside the sequential value)
    concurrent = None
    if args.concurrent_steps > 0:
        import threading
        ctxs = [ada.Context(0) for _ in cases]
        streams = [torch.cuda.Stream(device=dev) for _ in cases]
        cres = [None] * len(cases)

        def solve_one(k):
            name, A, B, kw, work, X, n = cases[k]
            with torch.cuda.stream(streams[k]):
                _, cres[k] = ada.solve(A, B, out=X, work=work, ctx=ctxs[k], **kw)

        def conc_step():
            ths = [threading.Thread(target=solve_one, args=(k,)) for k in range(len(cases))]
            for th in ths:
                th.start()
            for th in ths:
                th.join()

        conc_step()
        torch.cuda.synchronize()
        ct = []
        for _ in range(args.concurrent_steps):
            c0 = time.perf_counter()
            conc_step()
            ct.append(time.perf_counter() - c0)
        torch.cuda.synchronize()
        cworst = max(r.berr for r in cres)
        if not (cworst <= BERR_BAR) or any(r.route != info[c[0]].route for r, c in zip(cres, cases)):
            print(f"concurrent solves disagree with the sequential ones (max berr {cworst})", file=sys.stderr)
            sys.exit(1)
        concurrent = {"solves_per_s": round(len(cases) * len(ct) / sum(ct), 4),
                      "ms_per_step": round(sum(ct) / len(ct) * 1e3, 3),
                      "p50_step_ms": round(pct(ct, 50) * 1e3, 3), "max_berr": cworst, "streams": len(cases)}

    extensions = bench_extensions(args, cases, ctx, dev) if args.ext_steps > 0 else None

    cpu = None
    if not args.no_cpu and int(os.environ.get("RANK", "0")) == 0:
        cpu = cpu_baseline(host_cases)

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(total / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "single large systems: dense general n=8192, SPD n=8192, lower-triangular n=8192 "
                               "(off-diagonals / sqrt(n)), banded n=1e6 kl=ku=5 band layout, symmetric-indefinite "
                               f"n=4096; nrhs={args.nrhs}", "systems": names, "nrhs": args.nrhs},
        "tflops": round(flops_step * args.steps / total / 1e12, 4),
        "p50_step_ms": round(pct(step_times, 50) * 1e3, 3), "p99_step_ms": round(pct(step_times, 99) * 1e3, 3),
        "max_berr": worst_berr, "max_berr_oracle": max(oracle_eta.values()), "per_system": per_sys,
        "kernel_families": families,
        "kernel_families_from": "one untimed step with every kernel family timed",
        "roofline": roofline, "cpu_baseline": cpu, "concurrent": concurrent, "extensions": extensions,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
