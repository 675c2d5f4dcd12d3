"""Benchmark: static SABR surface calibration on one MI355X.

Workload (one step): 12 maturities {1m..10y} x 25 strikes (log-moneyness
+-0.6), beta in {0.5, 1.0}, each maturity fitted on its own: 24 calibrations
of 4096 synchronous annealing chains x 20000 iterations, float bulk
arithmetic with double near-the-money series, objective sums, accept
decisions and polish.  True
parameters are drawn uniformly in the box (seeded); the targets are the
library's double-precision vols at those parameters (noise-free).  The
requests are prepared once (validated, packed and copied to HBM); a step runs
the whole calibration on those resident inputs and brings the results back.
The same step from host arrays (sabr_calibrate_many) is reported beside it.

Prints one JSON line: calibrations/s (value), p50/p99 step latency, formula
evaluations/s, the annealing kernel's position against the VALU issue peak
(roofline), the FP64 oracle timed on the host (cpu_baseline), and a
Monte Carlo path-steps/s figure measured apart from the timed step.
"""
import argparse
import gc
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "calibrations/s + p50/p99 latency; MC path-steps/s; asymptotic-formula evals/s"
N_CHAINS, N_ITERS, CHAIN_LEN = 4096, 20000, 10
# Roofline of the ALU-bound kernels: the published FP32 vector peak of the
# chip, 157.3 TFLOP/s (256 CUs x 4 SIMDs x 32 FMA lanes per clock x 2 flops
# x 2.4 GHz), against the algorithmic FP32 flops of each unit of work, counting
# every FP32 add, multiply or FMA of the formula as an FMA (2 flops) and the
# transcendentals (exp, log, sqrt, reciprocal, sin, cos) as none:
#   static Hagan point evaluation       16 FP32 ops   = 32 flops (+ 3 transcendentals)
#   dynamic point evaluation             6 FP32 FMAs  = 12 flops
#   dynamic (chain, maturity) block     50 FP32 ops   = 100 flops (case I closed forms or series, + 2 exp)
#   Monte Carlo chain-path-step          7 FP32 ops   = 14 flops (+ 1 exp)
PEAK_FP32_TFLOPS = 157.3
FLOP_STATIC_PT, FLOP_DYN_PT, FLOP_DYN_BLOCK, FLOP_MC_STEP = 32, 12, 100, 14
TRANS_STATIC_PT = 3
ROOT_PROFILES = os.path.join(ROOT, "profiles")


def source_digest(files):
    """sha256 prefix of the kernel sources a counter summary was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_2407_20713_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


SA_SOURCES = ["sabr_dev.h", "sabr_formula.h", "sabr_sa.h", "kernels_formula.hip"]


def counter_summary(name, sources):
    """The machine-readable line of a committed counter summary under
    profiles/ (`counters: {...}`), or None when the kernel sources have
    changed since the counters were taken (its `sources` digest differs)."""
    path = os.path.join(ROOT_PROFILES, name)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("counters: "):
            d = json.loads(line[len("counters: "):])
            return d if d.get("sources") == source_digest(sources) else None
    return None


def build_requests(S, inputs, ctx, precision, polish=True):
    fits = inputs.surface_fits()
    gens, lb, ub = inputs.surface_true_params(len(fits))
    reqs, truths = [], []
    for k, g in enumerate(fits):
        beta = g.meta["beta"]
        mk = S.Market.from_grid(g)
        pb = S.Problem(S.SABR_STATIC, beta)
        while True:     # redraw until the surface is finite and positive
            x = inputs.draw_params(gens[k], lb, ub)
            _, vol = S.sabr_objective_batch(ctx, mk, pb, x[None, :], precision=S.SABR_FP64, want_model=True)
            if np.all(np.isfinite(vol)) and np.all(vol > 0):
                break
        req = S.Request(S.Market.from_grid(g, target=vol[0]), S.Problem(S.SABR_STATIC, beta, lb, ub),
                        precision=precision, n_chains=N_CHAINS, n_iters=N_ITERS, chain_len=CHAIN_LEN,
                        cooling=0.99 ** (1000.0 / N_ITERS), seed=0x5AB20000 + k, polish=polish)
        reqs.append(req)
        truths.append(x)
    return reqs, truths


def exact_solutions(x, beta, T, lb, ub):
    """The true parameters and, for beta = 1, the second exact fit of Hagan's
    formula (section 2.1) inside the box.  With rho and c = nu/alpha held,
    every vol of the maturity is z/x(z) (z = c ln(f/K)) times
    alpha + k alpha^3, k = T (rho c / 4 + (2 - 3 rho^2) c^2 / 24); for k < 0
    that cubic takes the truth's value again at the other positive root of
    a^2 + alpha a + alpha^2 + 1/k = 0, so that point fits the surface
    exactly too."""
    sols = [np.asarray(x, dtype=np.float64)]
    if beta != 1.0:
        return sols
    al, rho, nu = (float(v) for v in x)
    c = nu / al
    k = T * (rho * c / 4.0 + (2.0 - 3.0 * rho * rho) * c * c / 24.0)
    disc = -3.0 * al * al - 4.0 / k if k < 0 else -1.0
    if disc > 0:
        a2 = 0.5 * (-al + math.sqrt(disc))
        x2 = np.array([a2, rho, c * a2])
        if abs(a2 - al) > 1e-9 and np.all(x2 >= lb) and np.all(x2 <= ub):
            sols.append(x2)
    return sols


def recovery(results, truths, reqs):
    """Distance of each fit's result to the nearest exact solution of its
    noise-free surface; fits with two exact solutions are listed with the
    one the calibration returned."""
    err, two = 0.0, []
    for k, (r, x, q) in enumerate(zip(results, truths, reqs)):
        sols = exact_solutions(x, q.problem.beta, float(q.market.T[0]), q.problem.lb, q.problem.ub)
        d = [float(np.max(np.abs(r["x"] - s))) for s in sols]
        err = max(err, min(d))
        if len(sols) > 1:
            two.append({"fit": k, "T": float(q.market.T[0]), "truth": [round(float(v), 6) for v in x],
                        "other": [round(float(v), 6) for v in sols[1]],
                        "found": "truth" if d[0] <= d[1] else "other", "f": float(r["f"])})
    return err, two


def mc_path_steps(S, ctx, n_paths=1 << 24):
    """The paper's European call (Section 6.1: 123 steps of 1/250 y), case I
    parameters, float paths; path-steps per second of the pricing kernel."""
    S0 = K = 2257.37
    r, y, T = 0.018196, 0.034516, 0.495890
    f = S0 * math.exp((r - y) * T)
    from paper_2407_20713_amd import inputs
    g = inputs.make_grid([T], [[K]], f0=f, disc=[math.exp(-r * T)])
    pb = S.Problem(S.SABR_DYN_I, 1.0, x0=[0.393329, -1.0, 0.941565, 0.001, 1.246906])
    S.sabr_mc_price(ctx, S.Market.from_grid(g), pb, 1 << 16)
    S.sabr_ctx_timing(ctx, reset=True)
    t = time.perf_counter()
    p, se = S.sabr_mc_price(ctx, S.Market.from_grid(g), pb, n_paths)
    wall = time.perf_counter() - t
    ms, n, _ = S.sabr_ctx_timing(ctx, reset=True)
    steps = 123
    # the same call on antithetic pairs (a variance reduction the paper does
    # not use): its error against the plain scheme's on as many paths
    pa, sa = S.sabr_mc_price(ctx, S.Market.from_grid(g), pb, n_paths, scheme=S.SABR_MC_ANTITHETIC)
    ms_a, _, _ = S.sabr_ctx_timing(ctx, reset=True)
    return dict(workload="European call, case I, 2^24 paths x 123 steps, fp32", price=float(p[0]),
                std_err=float(se[0]), kernel_ms=ms, wall_ms=wall * 1e3,
                path_steps_per_s=n_paths * steps / (ms / 1e3),
                antithetic={"price": float(pa[0]), "std_err": float(sa[0]), "kernel_ms": ms_a,
                            "variance_ratio": float((se[0] / sa[0]) ** 2)})


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Host cores this process may use (at most 16, the CPU share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(reqs, gpu_results, sample_iters):
    """The FP64 oracle on the host: one fit of the same workload with 4096
    chains and `sample_iters` iterations on one core, scaled to full
    calibrations; then every usable core (one thread each, the oracle runs in
    C without the interpreter lock) on a fit of its own with half that many
    iterations at once, for the aggregate rate."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import oracle as O

    def one(k, iters):
        req = reqs[k % len(reqs)]
        m = req.market
        om = O.Market(m.T, m.fwd, m.offs, m.K, target=m.target)
        p = req.problem
        t = time.perf_counter()
        O.calibrate(om, O.STATIC, p.lb, p.ub, p.beta, N_CHAINS, iters, int(req.sa.seed),
                    cooling=req.sa.cooling, chain_len=CHAIN_LEN)
        return time.perf_counter() - t

    dt = one(5, sample_iters)
    per_cal = dt * (N_ITERS / sample_iters)
    n_thr = host_threads()
    it_all = max(sample_iters // 2, 10)
    with ThreadPoolExecutor(n_thr) as ex:
        t = time.perf_counter()
        times = list(ex.map(lambda k: one(k, it_all), range(n_thr)))
        wall = time.perf_counter() - t
    agg = n_thr / (wall * (N_ITERS / it_all))
    m = reqs[5].market
    return dict(value=agg, unit="calibrations/s", cores=n_thr, kind="oracle", cpu_model=cpu_model(),
                sample="%d threads at once, each one of the 24 fits (25 strikes) with %d chains x %d of %d "
                       "iterations, FP64, %.1f s wall (%.1f s of CPU), scaled by %d" % (
                           n_thr, N_CHAINS, it_all, N_ITERS, wall, sum(times), N_ITERS // it_all),
                single_core={"value": 1.0 / per_cal, "unit": "calibrations/s", "cores": 1,
                             "sample": "1 fit (T=%.3g), %d chains x %d of %d iterations, %.1f s, scaled by %d" % (
                                 m.T[0], N_CHAINS, sample_iters, N_ITERS, dt, N_ITERS // sample_iters),
                             "ns_per_point_eval": dt / (N_CHAINS * sample_iters * m.n_obs) * 1e9})


def fp32_vs_oracle(S, ctx, reqs, results):
    from oracle import oracle as O
    worst = 0.0
    for req, res in zip(reqs, results):
        m = req.market
        om = O.Market(m.T, m.fwd, m.offs, m.K)
        ref = O.model_vols(om, O.STATIC, res["x"], req.problem.beta)
        _, v32 = S.sabr_objective_batch(ctx, S.Market(m.T, m.fwd, m.offs, m.K), S.Problem(S.SABR_STATIC,
                                        req.problem.beta), res["x"][None, :], precision=S.SABR_FP32,
                                        want_model=True)
        worst = max(worst, float(np.max(np.abs(v32[0] - ref))))
    return worst


# --- other workloads (not the default line) ------------------------------------
def roofline(flops, kernel_s, kernel, launches, counters=None, units=None):
    """The dominant kernel against the FP32 vector peak: algorithmic flops of
    a launch over its average time; beside it, from the counter summary of
    the same kernel sources, the HBM traffic, the VALU issue rate and the FP32
    flops the hardware counted per unit of work (FMA = 2, every lane), scaled
    to this launch's `units`."""
    d = {"bound": "alu", "achieved": flops / kernel_s / 1e12, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
         "frac": flops / kernel_s / 1e12 / PEAK_FP32_TFLOPS, "traffic": None, "kernel": kernel,
         "avg_kernel_ms": kernel_s * 1e3, "launches": launches}
    if counters:
        d["traffic"] = counters.get("traffic_bytes_per_launch")
        d["valu_insts_per_simd_cycle"] = counters.get("valu_insts_per_simd_cycle")
        d["valu_busy_rocprof"] = counters.get("valu_busy_rocprof")
        per_unit = counters.get("executed_fp32_flops_per_unit")
        if per_unit is not None and units:
            d["executed_fp32_tflops"] = per_unit * units / kernel_s / 1e12
            d["executed_fp32_frac"] = d["executed_fp32_tflops"] / PEAK_FP32_TFLOPS
        d["counters_from"] = counters.get("file")
    return d


def bench_mc_calibration(S, inputs, ctx, args):
    """Monte Carlo objective calibration: 8 quarterly maturities x 15 strikes,
    static SABR (beta 0.7), 1024 chains x `iters` iterations x 65536 common
    paths, 250 steps per year, relative squared price errors; targets from a
    2^22-path FP64 run at the true parameters (Monte Carlo noise bounds the
    recovery), and, as the self-consistent variant, targets priced on the
    same 65536 common paths at the true parameters (the truth is then an
    exact minimum)."""
    g = inputs.mc_grid()
    xt = g.meta["x_true"]
    lb, ub = inputs.box(inputs.STATIC)
    iters = args.mc_iters
    tgt, _ = S.sabr_mc_price(ctx, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7, x0=xt), 1 << 22, 250,
                             g.meta["target_seed"], precision=S.SABR_FP64)
    _, same = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7), xt[None, :],
                                     kind=S.SABR_OBJ_MC, precision=S.SABR_FP32, n_paths=65536, steps_per_year=250,
                                     mc_seed=g.meta["mc_seed"], want_model=True)

    def run(target):
        req = S.Request(S.Market.from_grid(g, target=target), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                        kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=1024,
                        n_iters=iters, cooling=0.99 ** (1000.0 / 500), seed=0x5AB30001, n_paths=65536,
                        steps_per_year=250, mc_seed=g.meta["mc_seed"])
        S.sabr_ctx_enable_timing(ctx, True)
        S.sabr_ctx_timing(ctx, reset=True)
        t = time.perf_counter()
        res = S.sabr_calibrate(ctx, req)
        wall = time.perf_counter() - t
        ms, n, name = S.sabr_ctx_timing(ctx, reset=True)
        return res, wall, ms, n, name

    res, wall, ms, n, name = run(tgt)
    res_same, wall2, _, _, _ = run(same[0])
    m_max = 500
    cps = 1024 * 65536 * m_max * iters
    k_s = ms / 1e3 / max(n, 1)
    return {"metric": "MC path-steps/s", "value": cps / wall, "unit": "chain-path-steps/s",
            "kernel_chain_path_steps_per_s": cps / (ms / 1e3) if ms else None, "wall_s": wall,
            "calibrations_per_s": 1.0 / wall,
            "config": {"workload": "MC-objective calibration, 8 x 15 calls, 1024 chains x %d iterations x 65536 "
                                   "paths x 500 steps, FP32 paths" % iters},
            "roofline": roofline(1024 * 65536 * m_max * FLOP_MC_STEP, k_s, name, n,
                                 counter_summary("counters_mc_crn_kernel_mc_calibration.md",
                                                 ["sabr_dev.h", "sabr_mc.h", "kernels_mc.hip"]),
                                 units=1024 * 65536 * m_max),
            "param_error_vs_truth": float(np.max(np.abs(res["x"] - xt))), "f": res["f"],
            "self_consistent": {"param_error_vs_truth": float(np.max(np.abs(res_same["x"] - xt))),
                                "f": res_same["f"], "wall_s": wall2,
                                "targets": "FP32 prices on the same 65536 common paths at the truth"}}


def bench_surface_fp64(S, inputs, ctx, args):
    """The static surface workload in FP64 mode (every formula evaluation in
    double, the same fits, chains and iterations): one prepared batch, one
    warm-up run and two timed ones."""
    reqs, truths = build_requests(S, inputs, ctx, S.SABR_FP64)
    batch = S.sabr_batch_prepare(ctx, reqs)
    S.sabr_ctx_enable_timing(ctx, True)
    S.sabr_batch_run(batch, raw=True)
    S.sabr_ctx_timing(ctx, reset=True)
    reps = 2
    t = time.perf_counter()
    for _ in range(reps):
        S.sabr_batch_run(batch, raw=True)
    wall = (time.perf_counter() - t) / reps
    ms, n, name = S.sabr_ctx_timing(ctx, reset=True)
    results = S.sabr_batch_run(batch)
    S.sabr_batch_destroy(batch)
    err, _ = recovery(results, truths, reqs)
    pts = N_CHAINS * N_ITERS * sum(r.market.n_obs for r in reqs)
    k_s = ms / 1e3 / max(n, 1)
    return {"metric": "calibrations/s", "value": len(reqs) / wall, "unit": "calibrations/s",
            "ms_per_step": wall * 1e3, "kernel": name, "avg_kernel_ms": k_s * 1e3,
            "formula_evals_per_s": pts / k_s, "max_param_error_vs_exact_fit": err,
            "config": {"workload": "static SABR surface as the default line, FP64 throughout (24 fits x 4096 "
                                   "chains x 20000 iterations)"}}


def bench_dynamic(S, inputs, ctx, args):
    """Dynamic SABR case I, joint fit of 20 maturities x 20 strikes, 5
    parameters, 8192 chains x `iters` iterations, FP32 bulk, polish."""
    g = inputs.dynamic_surface()
    xt = g.meta["x_true"]
    lb, ub = inputs.box(inputs.DYN_I)
    _, vol = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(S.SABR_DYN_I, 0.7), xt[None, :],
                                    precision=S.SABR_FP64, want_model=True)
    iters = args.dyn_iters
    req = S.Request(S.Market.from_grid(g, target=vol[0]), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                    precision=S.SABR_FP32, n_chains=8192, n_iters=iters, cooling=0.99 ** (1000.0 / iters),
                    seed=0x5AB40001, polish=True)
    S.sabr_ctx_enable_timing(ctx, True)
    S.sabr_calibrate(ctx, req)
    S.sabr_ctx_timing(ctx, reset=True)
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        res = S.sabr_calibrate(ctx, req)
    wall = (time.perf_counter() - t) / reps
    ms, n, name = S.sabr_ctx_timing(ctx, reset=True)
    k_s = ms / 1e3 / max(n, 1)
    pts = 8192 * iters * g.n_obs
    flops = pts * FLOP_DYN_PT + 8192 * iters * g.n_mat * FLOP_DYN_BLOCK
    return {"metric": "asymptotic-formula evals/s", "value": pts / wall, "unit": "point-evals/s",
            "calibrations_per_s": 1.0 / wall, "wall_s": wall,
            "config": {"workload": "dynamic SABR case I, 20 x 20 joint fit, 8192 chains x %d iterations, FP32 "
                                   "bulk, FP64 polish" % iters},
            "roofline": roofline(flops, k_s, name, n,
                                 counter_summary("sa_kernel_dynamic_case1.md", SA_SOURCES), units=8192 * iters),
            "param_error_vs_truth": float(np.max(np.abs(res["x"] - xt))), "f": res["f"]}


def serving_requests(S, inputs, ctx, n, rate, seed, mc_paths):
    """Requests of the serving trace: 70 % static (256 chains x 2000), 20 %
    dynamic case I (512 x 4000), 10 % Monte Carlo (64 x 100 x mc_paths),
    targets = the library's FP64 model values at the drawn parameters plus
    N(0, 1e-4) vol noise (Monte Carlo: FP64 prices from another seed)."""
    trace = inputs.request_trace(n, rate, seed=seed)
    reqs = []
    for tr in trace:
        g = tr.grid
        if tr.kind == "mc":
            lb, ub = inputs.box(inputs.STATIC)
            tgt, _ = S.sabr_mc_price(ctx, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7, x0=tr.x_true),
                                     1 << 16, 250, tr.seed + 1, precision=S.SABR_FP32)
            tgt = np.maximum(tgt, 1e-8)
            req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                            kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=64,
                            n_iters=100, seed=tr.seed, n_paths=mc_paths, steps_per_year=250, mc_seed=tr.seed + 2)
        else:
            model = S.SABR_STATIC if tr.kind == "static" else S.SABR_DYN_I
            lb, ub = inputs.box(model)
            _, vol = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(model, 0.7), tr.x_true[None, :],
                                            precision=S.SABR_FP64, want_model=True)
            tgt = vol[0] + tr.noise
            chains, iters = (256, 2000) if tr.kind == "static" else (512, 4000)
            req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(model, 0.7, lb, ub),
                            precision=S.SABR_FP32, n_chains=chains, n_iters=iters, seed=tr.seed, polish=True)
        reqs.append(req)
    return trace, reqs


def serve(S, ctx, trace, reqs, rate_scale, max_slots, quantum):
    """Submit each request at its (scaled) arrival time; returns latencies (in
    completion order), the kind of request each one belongs to, the makespan
    and the server's statistics."""
    srv = S.Server(ctx, max_slots=max_slots, hbm_budget_bytes=8 << 30, quantum_levels=quantum)
    t0 = time.perf_counter()
    lat, kind, pending, i = [], [], 0, 0
    kind_of = {}
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and trace[i].arrival_s * rate_scale <= now:
            kind_of[srv.submit(reqs[i])] = trace[i].kind
            i += 1
            pending += 1
        for t, res, l in srv.poll(256, 500):
            lat.append(l)
            kind.append(kind_of.pop(t))
            pending -= 1
            if len(lat) % 200 == 0:
                print("served %d / %d" % (len(lat), len(reqs)), file=sys.stderr, flush=True)
    span = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    return np.array(lat), np.array(kind), span, st


def latency_by_kind(lat, kind):
    """p50 / p99 in ms of each kind of request present."""
    return {k: {"requests": int(np.sum(kind == k)), "p50_ms": float(np.percentile(lat[kind == k], 50) * 1e3),
                "p99_ms": float(np.percentile(lat[kind == k], 99) * 1e3)}
            for k in ("static", "dynamic", "mc") if np.any(kind == k)}


def bench_serving(S, inputs, ctx, args):
    """Config 5: capacity (every request submitted at once), then the trace's
    Poisson arrivals at a rate the server sustains (served rate within 5 % of
    the offered rate, found by trying 0.5 and then 0.35 of the capacity), and
    the first `serve_baseline` requests of the same arrivals served one
    sabr_calibrate call per request, first come first served."""
    n = args.serve_requests
    trace, reqs = serving_requests(S, inputs, ctx, n, 1.0, 0x5AB5, args.serve_paths)
    lat_b, _, span_b, st_b = serve(S, ctx, trace, reqs, 0.0, args.serve_slots, args.serve_quantum)
    capacity = n / span_b
    tried = []
    for frac in (0.5, 0.35):
        rate = frac * capacity
        lat_s, kind_s, span_s, st_s = serve(S, ctx, trace, reqs, 1.0 / rate, args.serve_slots, args.serve_quantum)
        offered = n / (trace[-1].arrival_s / rate)
        served = n / span_s
        tried.append({"fraction_of_capacity": frac, "offered_per_s": offered, "served_per_s": served,
                      "p50_ms": float(np.percentile(lat_s, 50) * 1e3),
                      "p99_ms": float(np.percentile(lat_s, 99) * 1e3),
                      "by_kind": latency_by_kind(lat_s, kind_s)})
        if served >= 0.95 * offered:
            break
    nb = min(args.serve_baseline, n)
    t0 = time.perf_counter()
    lat_1 = []
    for tr, r in zip(trace[:nb], reqs[:nb]):
        arr = tr.arrival_s / rate
        now = time.perf_counter() - t0
        if now < arr:
            time.sleep(arr - now)
        S.sabr_calibrate(ctx, r)
        lat_1.append(time.perf_counter() - t0 - arr)
        if len(lat_1) % 500 == 0:
            print("one-per-launch %d / %d" % (len(lat_1), nb), file=sys.stderr, flush=True)
    span_1 = time.perf_counter() - t0
    lat_1 = np.array(lat_1)
    kinds = {k: sum(1 for t in trace if t.kind == k) for k in ("static", "dynamic", "mc")}
    last = tried[-1]
    return {"metric": "calibrations/s + p50/p99 latency", "value": last["served_per_s"], "unit": "calibrations/s",
            "config": {"workload": "serving trace: %d requests, Poisson arrivals, 1-20 maturities x 5-41 strikes, "
                                   "mix %s, Monte Carlo %d paths" % (n, kinds, args.serve_paths),
                       "slots": args.serve_slots, "quantum_levels": args.serve_quantum},
            "capacity_calibrations_per_s": capacity,
            "sustained": dict(last, sustained=last["served_per_s"] >= 0.95 * last["offered_per_s"],
                              peak_active=st_s["peak_active"], peak_bytes=st_s["peak_bytes"], quanta=st_s["quanta"]),
            "rates_tried": tried,
            "one_request_per_launch": {"requests": nb, "offered_per_s": last["offered_per_s"],
                                       "calibrations_per_s": nb / span_1,
                                       "p50_ms": float(np.percentile(lat_1, 50) * 1e3),
                                       "p99_ms": float(np.percentile(lat_1, 99) * 1e3),
                                       "by_kind": latency_by_kind(lat_1, np.array([t.kind for t in trace[:nb]]))}}


def bench_copy(S, inputs, ctx, args):
    """Reference for the HBM byte counters: a plain device-to-device copy of
    a known size (read once, written once)."""
    import torch
    n = args.copy_mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = 10
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    return {"metric": "copy bandwidth", "value": 2 * n / dt / 1e9, "unit": "GB/s", "bytes_read": n,
            "bytes_written": n, "config": {"workload": "device copy of %d MiB" % args.copy_mib}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="surface",
                    choices=["surface", "surface_fp64", "mc_calibration", "dynamic", "serving", "copy"])
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--mc-iters", type=int, default=500)
    ap.add_argument("--dyn-iters", type=int, default=50000)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--serve-paths", type=int, default=16384)
    ap.add_argument("--serve-slots", type=int, default=1024)
    ap.add_argument("--serve-quantum", type=int, default=20)
    ap.add_argument("--serve-baseline", type=int, default=2000)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=2000)
    ap.add_argument("--no-mc", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="the static surface line only (no other configs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the calibration path is built and measured on a single "
              "MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    # No torch here (the copy reference aside): every library call below
    # returns only after the library's stream has finished, and without
    # torch the library binds to the HIP runtime under /opt/rocm, the one a
    # profiler attached to this process instruments.
    from paper_2407_20713_amd import inputs, sabr as S

    S.lib(bind_torch_runtime=args.workload == "copy")
    ctx = S.sabr_ctx_create(0)
    if args.workload != "surface":
        fn = {"mc_calibration": bench_mc_calibration, "dynamic": bench_dynamic, "serving": bench_serving,
              "copy": bench_copy, "surface_fp64": bench_surface_fp64}
        out = fn[args.workload](S, inputs, ctx, args)
        out.update({"n_gpus": 1, "data": "synthetic", "higher_is_better": True})
        ctx.close()
        print(json.dumps(out))
        return
    reqs, truths = build_requests(S, inputs, ctx, S.SABR_FP32)
    # The grids, schedules and launch plan are validated and copied to HBM once
    # (a prepared batch); a timed step is the whole calibration on them: grid
    # normalisation, annealing, polish and the results back on the host.
    batch = S.sabr_batch_prepare(ctx, reqs)
    S.sabr_ctx_enable_timing(ctx, True)
    for _ in range(args.warmup):
        S.sabr_batch_run(batch, raw=True)
    S.sabr_ctx_timing(ctx, reset=True)
    lat = []
    # Python's cyclic garbage collector is paused over the timed steps (as
    # timeit does), so that a collection of the interpreter's objects is not
    # charged to a step
    gc.collect()
    gc.disable()
    t_all = time.perf_counter()
    for _ in range(args.steps):
        t = time.perf_counter()
        S.sabr_batch_run(batch, raw=True)      # returns with the device idle
        lat.append(time.perf_counter() - t)
    total = time.perf_counter() - t_all
    gc.enable()
    kernel_ms, launches, kname = S.sabr_ctx_timing(ctx, reset=True)
    results = S.sabr_batch_run(batch)
    # the same calibrations from host arrays (validation, packing and the
    # host-to-device copies included in every call); reported beside the value
    n_host = min(args.steps, 3)
    t = time.perf_counter()
    for _ in range(n_host):
        host_res = S.sabr_calibrate_many(ctx, reqs)
    host_s = (time.perf_counter() - t) / max(n_host, 1)
    same = all(np.array_equal(a["x"], b["x"]) and a["f"] == b["f"] for a, b in zip(results, host_res))
    S.sabr_batch_destroy(batch)

    n_cal = len(reqs)
    pts = sum(r.market.n_obs for r in reqs)
    pt_evals = N_CHAINS * N_ITERS * pts            # per step (one sa_kernel launch)
    avg_kernel_s = kernel_ms / 1e3 / max(launches, 1)
    param_err, two_solutions = recovery(results, truths, reqs)
    lat_ms = np.array(lat) * 1e3
    rl = roofline(pt_evals * FLOP_STATIC_PT, avg_kernel_s, kname, launches,
                  counter_summary("counters_sa_kernel_static_surface.md", SA_SOURCES), units=pt_evals)
    rl["transcendentals_per_s"] = pt_evals * TRANS_STATIC_PT / avg_kernel_s
    out = {
        "metric": METRIC,
        "value": n_cal * args.steps / total,
        "unit": "calibrations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "static SABR surface: 12 maturities x 25 strikes, beta in {0.5, 1.0}, "
                               "24 single-maturity fits x 4096 chains x 20000 iterations, FP32 bulk, "
                               "FP64 near-ATM series, objective sums, decisions and polish",
                   "fits": n_cal, "chains": N_CHAINS, "iterations": N_ITERS, "chain_len": CHAIN_LEN,
                   "points_per_fit": 25},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99)),
                       "steps": [round(float(v), 2) for v in lat_ms]},
        "formula_evals_per_s": pt_evals * args.steps / total,
        "host_inputs": {"calibrations_per_s": n_cal / host_s, "ms_per_step": host_s * 1e3, "steps": n_host,
                        "identical_results": same},
        "max_param_error_vs_truth": param_err,
        "fits_with_two_exact_solutions": two_solutions,
        "roofline": rl,
    }
    if not args.no_mc:
        out["mc_path_steps"] = mc_path_steps(S, ctx)
    if not args.no_cpu_baseline:
        # the oracle leg: its timing, and its vols at the calibrated points
        # against the library's FP32 vols there
        cb = cpu_baseline(reqs, results, args.cpu_sample_iters)
        cb["fp32_vols_max_abs_error"] = fp32_vs_oracle(S, ctx, reqs, results)
        out["cpu_baseline"] = cb
    if not args.no_extra:
        print("static surface done; other configs follow", file=sys.stderr, flush=True)
        out["configs"] = {}
        for name, fn in (("surface_fp64", bench_surface_fp64), ("dynamic", bench_dynamic),
                         ("mc_calibration", bench_mc_calibration), ("serving", bench_serving)):
            out["configs"][name] = fn(S, inputs, ctx, args)
            print("%s done" % name, file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
