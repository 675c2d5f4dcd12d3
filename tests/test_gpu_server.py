"""GPU tests of the serving loop (sabr_server_*): each request's result is the
same alone, in a mix and for another quantum length (bitwise), results match
the oracle's calibration, admission respects the memory budget, and the
error paths (cancel, poll timeout, unsupported request) behave."""
import sys
import time

import numpy as np
import pytest

from paper_2407_20713_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2407_20713_amd import sabr
    sabr.lib()
    return sabr


@pytest.fixture(scope="module")
def ctx(S):
    c = S.sabr_ctx_create(0)
    yield c
    c.close()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def build_request(S, oracle, tr, n_chains, n_iters, mc_paths=512, polish=True):
    """A serving request from a trace entry (targets from the oracle)."""
    g = tr.grid
    m = oracle.Market(g.T, g.fwd, g.offs, g.K, disc=g.disc)
    if tr.kind == "static":
        tgt = oracle.model_vols(m, oracle.STATIC, tr.x_true, 0.7) + tr.noise
        lb, ub = inputs.box(inputs.STATIC)
        req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                        precision=S.SABR_FP32, n_chains=n_chains, n_iters=n_iters, seed=tr.seed, polish=polish)
    elif tr.kind == "dynamic":
        tgt = oracle.model_vols(m, oracle.DYN_I, tr.x_true, 0.7) + tr.noise
        lb, ub = inputs.box(inputs.DYN_I)
        req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                        precision=S.SABR_FP32, n_chains=n_chains, n_iters=n_iters, seed=tr.seed, polish=polish)
    else:
        tgt, _ = oracle.mc_prices(m, oracle.STATIC, tr.x_true, 0.7, mc_paths, 250, tr.seed + 1)
        tgt = np.maximum(tgt, 1e-6)
        lb, ub = inputs.box(inputs.STATIC)
        req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                        kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32,
                        n_chains=min(n_chains, 64), n_iters=max(4, n_iters // 50), seed=tr.seed,
                        n_paths=mc_paths, steps_per_year=50, mc_seed=tr.seed + 1)
    return req, m, tgt


def run_all(srv, reqs, timeout_s=120.0):
    tickets = [srv.submit(r) for r in reqs]
    got = {}
    t0 = time.time()
    while len(got) < len(tickets) and time.time() - t0 < timeout_s:
        for t, res, lat in srv.poll(64, 200000):
            got[t] = (res, lat)
    assert len(got) == len(tickets), "server did not finish in time"
    return [got[t] for t in tickets]


def small_trace(n, seed, max_mat=6):
    tr = inputs.request_trace(n, 1000.0, seed=seed, max_mat=max_mat, strike_range=(5, 15))
    return tr


def test_alone_equals_mix_and_quantum(S, ctx, oracle):
    trace = small_trace(18, 77)
    kinds = [t.kind for t in trace]
    say("kinds", kinds)
    probe_by_kind = {}
    for t in trace:
        probe_by_kind.setdefault(t.kind, t)
    assert set(probe_by_kind) == {"static", "dynamic", "mc"}
    reqs = [build_request(S, oracle, t, 128 if t.kind == "static" else 96, 300)[0] for t in trace]
    srv = S.Server(ctx, max_slots=32, quantum_levels=4)
    mix = run_all(srv, reqs)
    srv.close()
    for kind, t in probe_by_kind.items():
        i = trace.index(t)
        srv1 = S.Server(ctx, max_slots=8, quantum_levels=7)
        alone = run_all(srv1, [reqs[i]])[0][0]
        srv1.close()
        a, b = alone, mix[i][0]
        say(kind, "alone", a["x"][:5], a["f"], "mix", b["x"][:5], b["f"])
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["x"], b["x"]) and a["f"] == b["f"] and a["n_accept"] == b["n_accept"]


def test_server_result_matches_oracle_calibration(S, ctx, oracle):
    """A static request served in FP32 with polish reaches the same least-squares
    point as the oracle's FP64 calibration (both polished)."""
    trace = small_trace(30, 5)
    t = next(x for x in trace if x.kind == "static")
    req, m, tgt = build_request(S, oracle, t, 128, 600)
    srv = S.Server(ctx, max_slots=8, quantum_levels=10)
    res = run_all(srv, [req])[0][0]
    srv.close()
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 128, 600, t.seed, polish=True)
    say("server", res["x"][:3], res["f"], "oracle", ref["x"], ref["f"])
    np.testing.assert_allclose(res["x"][:3], ref["x"], atol=1e-3)
    assert res["f"] <= ref["f"] * (1 + 1e-6) + 1e-14


def test_budget_admission(S, ctx, oracle):
    """With room for about two requests at a time every request still
    completes and the arena never holds more than the budget."""
    trace = [t for t in small_trace(40, 9) if t.kind == "static"][:6]
    reqs = [build_request(S, oracle, t, 128, 200)[0] for t in trace]
    budget = 2 * 1024 * 1024
    srv = S.Server(ctx, max_slots=16, hbm_budget_bytes=budget, quantum_levels=5)
    out = run_all(srv, reqs)
    st = srv.stats()
    srv.close()
    say("stats", st)
    assert all(r["status"] == 0 for r, _ in out)
    assert st["peak_bytes"] <= budget
    assert st["completed"] == len(reqs)


def test_cancel_timeout_and_rejection(S, ctx, oracle):
    srv = S.Server(ctx, max_slots=4, quantum_levels=2)
    assert srv.poll(4, 1000) == []          # nothing submitted: times out
    trace = [t for t in small_trace(40, 11) if t.kind == "static"][:3]
    reqs = [build_request(S, oracle, t, 128, 4000)[0] for t in trace]
    tickets = [srv.submit(r) for r in reqs]
    srv.cancel(tickets[1])
    got = {}
    t0 = time.time()
    while len(got) < 3 and time.time() - t0 < 120:
        for t, res, lat in srv.poll(8, 200000):
            got[t] = res
    assert got[tickets[1]]["status"] == S.SABR_E_CANCELLED
    assert got[tickets[0]]["status"] == 0 and got[tickets[2]]["status"] == 0
    # FP64 requests are served by sabr_calibrate, not by the server
    bad = build_request(S, oracle, trace[0], 64, 100)[0]
    bad.obj.precision = S.SABR_FP64
    with pytest.raises(S.SabrError) as e:
        srv.submit(bad)
    assert e.value.code == S.SABR_E_INVAL
    srv.close()


def test_monte_carlo_lds_classes_alone_equals_mix(S, ctx, oracle):
    """Monte Carlo requests of small, middle and large option counts (up to
    96, 256 and 600 options, whose path blocks share one launch)
    give bitwise the same result alone and together (for two quantum
    lengths)."""
    reqs = []
    for k, (n_mat, n_k) in enumerate(((4, 15), (8, 25), (12, 41))):
        T = [0.25 * (i + 1) for i in range(n_mat)]
        g = inputs.make_grid(T, [np.exp(np.linspace(-0.3, 0.3, n_k))] * n_mat, f0=1.0)
        m = oracle.Market(g.T, g.fwd, g.offs, g.K, disc=g.disc)
        tgt, _ = oracle.mc_prices(m, oracle.STATIC, [0.25, -0.2, 0.4], 0.7, 256, 50, 900 + k)
        tgt = np.maximum(tgt, 1e-6)
        lb, ub = inputs.box(inputs.STATIC)
        reqs.append(S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                              kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32,
                              n_chains=24, n_iters=6, seed=40 + k, n_paths=300, steps_per_year=50,
                              mc_seed=70 + k))
        say("class case", k, "options", g.n_obs)
    srv = S.Server(ctx, max_slots=16, quantum_levels=3)
    mix = run_all(srv, reqs)
    srv.close()
    for i, r in enumerate(reqs):
        srv1 = S.Server(ctx, max_slots=16, quantum_levels=5)
        alone = run_all(srv1, [r])[0][0]
        srv1.close()
        a, b = alone, mix[i][0]
        say("mc class", i, a["x"][:3], a["f"], b["f"])
        assert a["status"] == 0 and b["status"] == 0
        assert np.array_equal(a["x"], b["x"]) and a["f"] == b["f"] and a["n_accept"] == b["n_accept"]
        assert np.isfinite(a["f"]) and a["f"] >= 0.0


def test_second_wave_joins_running_requests(S, ctx, oracle):
    """Continuous batching: with few slots and room in the memory budget for
    about two requests, a second wave submitted while the first is on the
    device (quanta already run) is admitted as slots and memory free up, and
    every result of both waves is bitwise the one the request gets alone."""
    trace = [t for t in small_trace(60, 21) if t.kind == "static"][:8]
    reqs = [build_request(S, oracle, t, 128, 1500)[0] for t in trace]
    srv = S.Server(ctx, max_slots=4, hbm_budget_bytes=2 * 1024 * 1024, quantum_levels=5)
    first = [srv.submit(r) for r in reqs[:4]]
    t0 = time.time()
    while srv.stats()["quanta"] == 0 and time.time() - t0 < 60:
        time.sleep(0.001)
    st = srv.stats()
    say("before second wave", st)
    assert st["quanta"] > 0 and st["completed"] < 4
    second = [srv.submit(r) for r in reqs[4:]]
    got = {}
    t0 = time.time()
    while len(got) < len(reqs) and time.time() - t0 < 120:
        for t, res, lat in srv.poll(16, 200000):
            got[t] = res
    st = srv.stats()
    srv.close()
    say("after", st)
    assert len(got) == len(reqs)
    for r, t in zip(reqs, first + second):
        srv1 = S.Server(ctx, max_slots=4, quantum_levels=5)
        alone = run_all(srv1, [r])[0][0]
        srv1.close()
        b = got[t]
        assert alone["status"] == 0 and b["status"] == 0
        assert np.array_equal(alone["x"], b["x"]) and alone["f"] == b["f"] and alone["n_accept"] == b["n_accept"]


def test_served_dynamic_request_matches_oracle_calibration(S, ctx, oracle):
    """A dynamic (case I) request served in FP32 with polish reaches the
    oracle's polished FP64 calibration to 1e-3."""
    trace = small_trace(40, 6)
    t = next(x for x in trace if x.kind == "dynamic" and x.grid.n_mat >= 3)
    req, m, tgt = build_request(S, oracle, t, 256, 2000)
    srv = S.Server(ctx, max_slots=8, quantum_levels=10)
    res = run_all(srv, [req])[0][0]
    srv.close()
    m.target = tgt
    lb, ub = inputs.box(inputs.DYN_I)
    ref = oracle.calibrate(m, oracle.DYN_I, lb, ub, 0.7, 256, 2000, t.seed, polish=True)
    say("served dynamic", res["x"][:5], res["f"], "oracle", ref["x"], ref["f"])
    np.testing.assert_allclose(res["x"][:5], ref["x"], atol=1e-3)
    assert res["f"] <= ref["f"] * (1 + 1e-6) + 1e-14


def test_served_monte_carlo_request_follows_oracle(S, ctx, oracle):
    """A Monte Carlo request served on the slot kernels (8 chains x 20
    iterations x 512 common paths) takes the oracle's accept decisions."""
    g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    m = oracle.Market(g.T, g.fwd, g.offs, g.K, disc=g.disc)
    tgt, _ = oracle.mc_prices(m, oracle.STATIC, [0.2, -0.3, 0.5], 0.7, 512, 250, 4242)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8,
                    n_iters=20, seed=3, n_paths=512, steps_per_year=250, mc_seed=4242)
    srv = S.Server(ctx, max_slots=16, quantum_levels=3)
    res = run_all(srv, [req])[0][0]
    srv.close()
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 8, 20, 3, weighting=oracle.RELATIVE,
                           objective=oracle.OBJ_MC, mc_paths=512, mc_steps_per_year=250, mc_seed=4242)
    say("served mc", res["x"][:3], res["n_accept"], "oracle", ref["x"], ref["n_accept"])
    assert res["status"] == 0 and res["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(res["x"][:3], ref["x"], atol=1e-12)
    assert abs(res["f"] - ref["f"]) <= 1e-3 * ref["f"]


def test_served_monte_carlo_at_the_path_limit(S, ctx, oracle):
    """A served Monte Carlo request of 131072 paths, the most a slot takes
    (512 path blocks of 256 paths: each lane adds 256 payoffs in float).  Its
    objective at the parameters it returns is the oracle's FP64 objective on
    the same common paths, within what a price error of 5e-5 relative plus
    1e-7 allows (the float path scheme's bound in the price parity tests):
    |f32 - f| <= sum_i (2 |e_i| d_i + d_i^2) w_i."""
    g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    m = oracle.Market(g.T, g.fwd, g.offs, g.K, disc=g.disc)
    n_paths, spy, mc_seed = 131072, 50, 777
    tgt, _ = oracle.mc_prices(m, oracle.STATIC, [0.2, -0.3, 0.5], 0.7, n_paths, spy, mc_seed + 1)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8,
                    n_iters=4, seed=5, n_paths=n_paths, steps_per_year=spy, mc_seed=mc_seed)
    srv = S.Server(ctx, max_slots=16, quantum_levels=3)
    res = run_all(srv, [req])[0][0]
    srv.close()
    assert res["status"] == 0
    x = np.asarray(res["x"][:3])
    ref_f = oracle.objective_mc(m, oracle.STATIC, x, 0.7, n_paths, spy, mc_seed, weighting=oracle.RELATIVE)
    price, _ = oracle.mc_prices(m, oracle.STATIC, x, 0.7, n_paths, spy, mc_seed)
    d = 5e-5 * np.abs(price) + 1e-7
    tol = float(np.sum((2 * np.abs(price - tgt) * d + d ** 2) / tgt ** 2))
    say("served mc at the path limit", x, res["f"], "oracle", ref_f, "tol", tol)
    assert np.isfinite(ref_f) and abs(res["f"] - ref_f) <= tol


def test_served_monte_carlo_path_limit(S, ctx, oracle):
    """A served Monte Carlo request adds at most 256 payoffs per lane in
    float: more than 256 x 512 paths is refused (sabr_calibrate takes it)."""
    g = inputs.make_grid([0.25], [np.exp(np.linspace(-0.2, 0.2, 3))], f0=1.0)
    lb, ub = inputs.box(inputs.STATIC)
    srv = S.Server(ctx, max_slots=16, quantum_levels=3)
    req = S.Request(S.Market.from_grid(g, target=np.full(3, 0.05)), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8,
                    n_iters=4, seed=3, n_paths=131073, steps_per_year=50, mc_seed=1)
    with pytest.raises(S.SabrError) as e:
        srv.submit(req)
    assert e.value.code == S.SABR_E_INVAL
    req.mc.n_paths = 131072
    srv.submit(req)
    srv.close()
