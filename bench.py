"""Benchmark: static SABR surface calibration on one MI355X.

Workload (one step): 12 maturities {1m..10y} x 25 strikes (log-moneyness
+-0.6), beta in {0.5, 1.0}, each maturity fitted on its own: 24 calibrations
of 4096 synchronous annealing chains x 20000 iterations, float bulk
arithmetic with double objective sums, accept decisions and polish.  True
parameters are drawn uniformly in the box (seeded); the targets are the
library's double-precision vols at those parameters (noise-free).

Prints one JSON line: calibrations/s (value), p50/p99 step latency, formula
evaluations/s, the annealing kernel's position against the VALU issue peak
(roofline), the FP64 oracle timed on the host (cpu_baseline), and a
Monte Carlo path-steps/s figure measured apart from the timed step.
"""
import argparse
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
# VALU issue peak of the chip in float lane-op slots: 256 CUs x 4 SIMDs x 32
# lanes per clock x 2.4 GHz = 78.64 T/s (the published 157.3 TFLOP/s FP32
# counts an FMA as two flops).  A double op takes 2 slots, a transcendental
# (exp, log, sqrt, rcp, sin, cos) 4.
PEAK_VALU_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
# Algorithmic slots of one float Hagan point evaluation (z, s, x(z), z/x,
# T-correction, vol, double residual and accumulation): 21 float ops, 3
# transcendentals, 3 double ops = 21 + 12 + 6 = 39; and of one annealing
# iteration outside the point loop (Philox4x32-10 with 20 32x32->64 multiplies
# at quarter rate, the double proposal and the Metropolis test with its
# double exp and division): ~200 slots.  Derivation in the design doc.
SLOTS_PER_PT_EVAL = 39
SLOTS_SA_PER_ITER = 200


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
    return dict(workload="European call, case I, 2^24 paths x 123 steps, fp32", price=float(p[0]),
                std_err=float(se[0]), kernel_ms=ms, wall_ms=wall * 1e3,
                path_steps_per_s=n_paths * steps / (ms / 1e3))


def cpu_baseline(reqs, gpu_results, sample_iters):
    """The FP64 oracle on one host core: one fit of the same workload with
    4096 chains and `sample_iters` iterations, scaled to full calibrations.
    Also reports the largest vol difference between the GPU's float vols and
    the oracle's double vols at the GPU's calibrated parameters."""
    from oracle import oracle as O
    req = reqs[5]
    m = req.market
    om = O.Market(m.T, m.fwd, m.offs, m.K, target=m.target)
    p = req.problem
    t = time.perf_counter()
    O.calibrate(om, O.STATIC, p.lb, p.ub, p.beta, N_CHAINS, sample_iters, int(req.sa.seed),
                cooling=req.sa.cooling, chain_len=CHAIN_LEN)
    dt = time.perf_counter() - t
    per_cal = dt * (N_ITERS / sample_iters)
    return dict(value=1.0 / per_cal, unit="calibrations/s", cores=1, kind="oracle",
                sample="1 of the 24 fits (25 strikes, T=%.3g), %d chains x %d of %d iterations, FP64, "
                       "%.1f s measured, scaled by %d" % (m.T[0], N_CHAINS, sample_iters, N_ITERS, dt,
                                                           N_ITERS // sample_iters),
                ns_per_point_eval=dt / (N_CHAINS * sample_iters * m.n_obs) * 1e9)


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=2000)
    ap.add_argument("--no-mc", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the calibration path is built and measured on a single "
              "MI355X; --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_20713_amd import inputs, sabr as S

    S.lib()
    ctx = S.sabr_ctx_create(0)
    reqs, truths = build_requests(S, inputs, ctx, S.SABR_FP32)
    S.sabr_ctx_enable_timing(ctx, True)
    for _ in range(args.warmup):
        S.sabr_calibrate(ctx, reqs)
    S.sabr_ctx_timing(ctx, reset=True)
    lat = []
    torch.cuda.synchronize()
    t_all = time.perf_counter()
    results = None
    for _ in range(args.steps):
        t = time.perf_counter()
        results = S.sabr_calibrate(ctx, reqs)
        lat.append(time.perf_counter() - t)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_all
    kernel_ms, launches, kname = S.sabr_ctx_timing(ctx, reset=True)

    n_cal = len(reqs)
    pts = sum(r.market.n_obs for r in reqs)
    pt_evals = N_CHAINS * N_ITERS * pts            # per step
    avg_kernel_s = kernel_ms / 1e3 / max(launches, 1)
    slots = pt_evals * SLOTS_PER_PT_EVAL + n_cal * N_CHAINS * N_ITERS * SLOTS_SA_PER_ITER
    achieved = slots / avg_kernel_s / 1e12
    param_err = max(float(np.max(np.abs(r["x"] - x))) for r, x in zip(results, truths))
    lat_ms = np.array(lat) * 1e3
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
                               "FP64 sums/decisions/polish",
                   "fits": n_cal, "chains": N_CHAINS, "iterations": N_ITERS, "chain_len": CHAIN_LEN,
                   "points_per_fit": 25},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "formula_evals_per_s": pt_evals * args.steps / total,
        "max_param_error_vs_truth": param_err,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "Tops/s",
                     "frac": achieved / PEAK_VALU_TOPS, "traffic": None,
                     "kernel": kname, "avg_kernel_ms": avg_kernel_s * 1e3, "launches": launches},
    }
    if not args.no_mc:
        out["mc_path_steps"] = mc_path_steps(S, ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(reqs, results, args.cpu_sample_iters)
        out["max_vol_error_fp32_vs_oracle"] = fp32_vs_oracle(S, ctx, reqs, results)
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
