"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Tolerances (stated once, used below):
  formula objective, FP64 mode : |df| <= 1e-12 f + 1e-14 sqrt(f S), S = sum w target^2
                                 (rounding of the model vols bounds |df| by ~eps sqrt(f S));
  model vols, FP64 mode        : 1e-13 relative + 1e-15 absolute (case II quadrature: 1e-10 relative);
  model vols, FP32 mode        : 2e-5 absolute vol;
  Monte Carlo prices, FP32     : 5e-5 relative on identical normals (plus 1e-7 absolute
                                 for prices of deep out-of-the-money strikes near 0);
  Monte Carlo prices, FP64     : 1e-9 relative;
  calibrated parameters        : 1e-3.
"""
import math
import sys

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


def omkt(oracle, g, target=None):
    return oracle.Market(g.T, g.fwd, g.offs, g.K, target=target, disc=g.disc)


def random_params(model, n, seed, beta_free=False):
    rng = np.random.default_rng(seed)
    lb, ub = inputs.box(model, beta_free)
    if model == inputs.DYN_II:
        lb = lb.copy(); ub = ub.copy()
        lb[5:9] *= 0.2; ub[5:9] *= 0.2     # mostly feasible case II vectors
    X = lb + (ub - lb) * rng.random((n, len(lb)))
    if model != inputs.STATIC:
        X[: n // 4, 3:5] *= 1e-3           # small rate * maturity: the series branch
    return X


def ragged_grid():
    """3 maturities with 7, 1 and 30 strikes (ragged rows, more than one tile)."""
    return inputs.make_grid([0.1, 1.3, 6.0], [np.exp(np.linspace(-0.4, 0.5, 7)), [1.02],
                                              np.exp(np.linspace(-0.7, 0.6, 30))], f0=1.3)


def objective_tol(f, S_):
    return 1e-12 * f + 1e-14 * np.sqrt(f * S_)


# --- formula objective -----------------------------------------------------------------
@pytest.mark.parametrize("formula", [0, 1, 2])
@pytest.mark.parametrize("beta_free", [False, True])
def test_static_objective_fp64(S, ctx, oracle, formula, beta_free):
    g = ragged_grid()
    say("static fp64 formula", formula, "beta_free", beta_free)
    X = random_params(inputs.STATIC, 300, 11 + formula, beta_free)
    beta = 0.6
    xt = np.array([0.25, -0.4, 0.7] + ([0.6] if beta_free else []))
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, xt, beta, beta_free, formula) + 1e-3
    m.target = tgt
    mk = S.Market.from_grid(g, target=tgt)
    pb = S.Problem(S.SABR_STATIC, beta, beta_free=beta_free)
    f, mod = S.sabr_objective_batch(ctx, mk, pb, X, formula=formula, precision=S.SABR_FP64, want_model=True)
    for i in range(len(X)):
        ref_v = oracle.model_vols(m, oracle.STATIC, X[i], beta, beta_free, formula)
        ref_f = oracle.objective_formula(m, oracle.STATIC, X[i], beta, beta_free, formula)
        ok = np.isfinite(ref_v) & (ref_v > 0)
        np.testing.assert_allclose(mod[i][ok], ref_v[ok], rtol=1e-13, atol=1e-15)
        if np.isfinite(ref_f):
            assert abs(f[i] - ref_f) <= objective_tol(ref_f, np.sum(tgt ** 2)), (i, f[i], ref_f)
        else:
            assert f[i] == np.inf


@pytest.mark.parametrize("formula", [0, 1, 2])
def test_static_objective_fp32(S, ctx, oracle, formula):
    g = ragged_grid()
    say("static fp32 formula", formula)
    X = random_params(inputs.STATIC, 400, 21 + formula)
    beta = 0.7
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.2, -0.3, 0.5], beta, False, formula)
    mk = S.Market.from_grid(g, target=tgt)
    pb = S.Problem(S.SABR_STATIC, beta)
    _, mod = S.sabr_objective_batch(ctx, mk, pb, X, formula=formula, precision=S.SABR_FP32, want_model=True)
    worst = 0.0
    for i in range(len(X)):
        ref_v = oracle.model_vols(m, oracle.STATIC, X[i], beta, False, formula)
        ok = np.isfinite(ref_v) & (ref_v > 0) & (ref_v < 5)
        worst = max(worst, np.max(np.abs(mod[i][ok] - ref_v[ok])) if ok.any() else 0.0)
    say("worst abs vol error fp32", worst)
    assert worst < 2e-5


@pytest.mark.parametrize("formula", [0, 1])
@pytest.mark.parametrize("weighting", [0, 1])
def test_static_objective_fp32_values(S, ctx, oracle, formula, weighting):
    """FP32 objective values without model output (the annealing's float
    loop: vols and residuals in float, their squares summed in double)
    against the oracle's FP64
    objective, within what a vol error of delta = 2e-5 allows:
    |f32 - f| <= sum_i (2 |e_i| delta + delta^2) w_i + 1e-6 f.  Ragged rows
    and strikes at and next to the forward (the near-the-money series)."""
    K0 = np.exp(np.linspace(-0.4, 0.5, 7))
    K1 = 1.3 * np.exp(np.array([-1e-2, -1e-4, -1e-7, 0.0, 1e-7, 1e-4, 1e-2]))
    K2 = np.exp(np.linspace(-0.7, 0.6, 30))
    g = inputs.make_grid([0.1, 1.3, 6.0], [K0, K1, K2], f0=1.3)
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.25, -0.4, 0.7], 0.6, False, formula) + 2e-3
    m.target = tgt
    X = random_params(inputs.STATIC, 300, 61 + formula)
    f, _ = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.6), X,
                                  formula=formula, weighting=weighting, precision=S.SABR_FP32)
    w = np.ones_like(tgt) if weighting == 0 else 1.0 / tgt ** 2
    delta, n_checked = 2e-5, 0
    for i in range(len(X)):
        ref_f = oracle.objective_formula(m, oracle.STATIC, X[i], 0.6, False, formula, weighting)
        ref_v = oracle.model_vols(m, oracle.STATIC, X[i], 0.6, False, formula)
        if not (np.isfinite(ref_f) and np.all(np.isfinite(ref_v)) and np.all((ref_v > 0.01) & (ref_v < 5))):
            continue
        tol = np.sum((2 * np.abs(tgt - ref_v) * delta + delta ** 2) * w) + 1e-6 * ref_f
        assert abs(f[i] - ref_f) <= tol, (i, f[i], ref_f, tol)
        n_checked += 1
    assert n_checked > 100


def test_static_near_the_money_island(S, ctx, oracle):
    """Strikes within 1e-7..1e-2 of the forward, where z/x(z) cancels."""
    K = 1.0 * np.exp(np.array([-1e-2, -1e-4, -1e-7, 0.0, 1e-7, 1e-4, 1e-2]))
    g = inputs.make_grid([0.5], [K])
    m = omkt(oracle, g)
    X = random_params(inputs.STATIC, 200, 5)
    for prec, tol in ((S.SABR_FP64, 1e-13), (S.SABR_FP32, 2e-5)):
        _, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.5), X,
                                        precision=prec, want_model=True)
        for i in range(len(X)):
            ref = oracle.model_vols(m, oracle.STATIC, X[i], 0.5)
            if prec == S.SABR_FP64:
                np.testing.assert_allclose(mod[i], ref, rtol=tol)
            else:
                assert np.max(np.abs(mod[i] - ref)) < tol


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("beta_free", [False, True])
def test_dynamic_case1_objective(S, ctx, oracle, prec, beta_free):
    g = inputs.dynamic_surface(n_mat=20, n_strikes=20)
    say("case I prec", prec, "beta_free", beta_free)
    m = omkt(oracle, g)
    xt = list(g.meta["x_true"]) + ([0.7] if beta_free else [])
    tgt = oracle.model_vols(m, oracle.DYN_I, xt, 0.7, beta_free)
    m.target = tgt
    X = random_params(inputs.DYN_I, 256, 31, beta_free)
    f, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt),
                                    S.Problem(S.SABR_DYN_I, 0.7, beta_free=beta_free), X, precision=prec,
                                    want_model=True)
    worst = 0.0
    for i in range(len(X)):
        ref_v = oracle.model_vols(m, oracle.DYN_I, X[i], 0.7, beta_free)
        ok = np.isfinite(ref_v) & (ref_v > 0) & (ref_v < 5)
        if prec == S.SABR_FP64:
            np.testing.assert_allclose(mod[i][ok], ref_v[ok], rtol=1e-13, atol=1e-15)
            ref_f = oracle.objective_formula(m, oracle.DYN_I, X[i], 0.7, beta_free)
            if np.isfinite(ref_f):
                assert abs(f[i] - ref_f) <= objective_tol(ref_f, np.sum(tgt ** 2))
        else:
            worst = max(worst, np.max(np.abs(mod[i][ok] - ref_v[ok])) if ok.any() else 0.0)
    if prec == S.SABR_FP32:
        say("worst case I fp32", worst)
        assert worst < 2e-5


@pytest.mark.parametrize("prec", [0, 1])
def test_dynamic_case2_objective(S, ctx, oracle, prec):
    g = inputs.make_grid([0.25, 1.0, 3.0], [np.exp(np.linspace(-0.4, 0.4, 5))] * 3)
    m = omkt(oracle, g)
    X = random_params(inputs.DYN_II, 24, 41)
    _, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(S.SABR_DYN_II, 0.7), X,
                                    precision=prec, want_model=True)
    for i in range(len(X)):
        if not oracle.case2_feasible(X[i], 3.0):
            continue
        ref_v = oracle.model_vols(m, oracle.DYN_II, X[i], 0.7)
        ok = np.isfinite(ref_v) & (ref_v > 0) & (ref_v < 5)
        if prec == S.SABR_FP64:
            np.testing.assert_allclose(mod[i][ok], ref_v[ok], rtol=1e-10)
        else:
            assert np.max(np.abs(mod[i][ok] - ref_v[ok])) < 2e-5


def test_objective_edge_cases(S, ctx):
    g = inputs.single_smile()
    mk = S.Market.from_grid(g, target=np.full(15, 0.2))
    pb = S.Problem(S.SABR_STATIC, 0.7)
    f, _ = S.sabr_objective_batch(ctx, mk, pb, np.zeros((0, 3)))
    assert len(f) == 0
    # a model vol that is not positive gives +inf
    f, _ = S.sabr_objective_batch(ctx, mk, pb, np.array([[0.2, -0.3, 0.5], [1e-9, 0.99, 2.0]]))
    assert np.isfinite(f[0])
    # invalid inputs are rejected with SABR_E_INVAL and a message
    bad = S.Market(g.T, g.fwd, [0, 0], g.K[:0], target=np.zeros(0))
    with pytest.raises(S.SabrError) as e:
        S.sabr_objective_batch(ctx, bad, pb, np.array([[0.2, -0.3, 0.5]]))
    assert e.value.code == S.SABR_E_INVAL
    with pytest.raises(S.SabrError) as e:
        S.sabr_objective_batch(ctx, mk, S.Problem(S.SABR_STATIC, 1.5), np.array([[0.2, -0.3, 0.5]]))
    assert e.value.code == S.SABR_E_INVAL


def test_objective_device_arrays(S, ctx, oracle):
    """X and f as torch tensors in HBM stay on the device."""
    import torch
    g = inputs.single_smile()
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.2, -0.3, 0.5], 0.7)
    X = random_params(inputs.STATIC, 1000, 3)
    Xd = torch.tensor(X, device="cuda", dtype=torch.float64)
    f, _ = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7), Xd,
                                  precision=S.SABR_FP64)
    torch.cuda.synchronize()
    assert f.is_cuda
    fh, _ = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7), X,
                                   precision=S.SABR_FP64)
    np.testing.assert_array_equal(f.cpu().numpy(), fh)


# --- Monte Carlo -------------------------------------------------------------------------
MC_CASES = [
    ("static", inputs.STATIC, [0.3, -0.5, 0.8], 0.7),
    ("case I", inputs.DYN_I, [0.393329, -1.0, 0.941565, 0.001, 1.246906], 1.0),
    ("case II", inputs.DYN_II, [0.398436, -0.964678, 1.285129, 0.0, 2.059560, 0.101632, -0.086294, 0.0,
                                1.302296], 0.999579),
]


@pytest.mark.parametrize("name,model,x,beta", MC_CASES)
@pytest.mark.parametrize("prec", [1, 0])
def test_mc_price_identical_normals(S, ctx, oracle, name, model, x, beta, prec):
    say("mc price", name, "prec", prec)
    g = inputs.make_grid([0.25, 0.5, 1.0], [np.exp(np.linspace(-0.3, 0.3, 5))] * 3, f0=1.0,
                         disc=[0.99, 0.98, 0.96])
    m = omkt(oracle, g)
    n_paths = 3000          # 12 tiles of 256 with a ragged last one
    ref, se = oracle.mc_prices(m, model, x, beta, n_paths, 250, 0xC0FFEE)
    got, gse = S.sabr_mc_price(ctx, S.Market.from_grid(g), S.Problem(model, beta, x0=x), n_paths, 250, 0xC0FFEE,
                               precision=prec)
    if prec == S.SABR_FP32:
        np.testing.assert_allclose(got, ref, rtol=5e-5, atol=1e-7)
    else:
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(gse, se, rtol=1e-6)


def test_mc_price_printed_case_full_size(S, ctx):
    """The paper's European call (2^20 paths, 123 steps): both dynamic rows land
    within 3 combined standard errors of the printed prices (sampled
    property at the benchmark size; parity with the oracle is above)."""
    S0 = K = 2257.37
    r, y, T = 0.018196, 0.034516, 0.495890
    f = S0 * math.exp((r - y) * T)
    g = inputs.make_grid([T], [[K]], f0=f, disc=[math.exp(-r * T)])
    for (name, model, x, beta), printed in zip(MC_CASES[1:], (222.434009, 224.653642)):
        p, se = S.sabr_mc_price(ctx, S.Market.from_grid(g), S.Problem(model, beta, x0=x), 1 << 20, 250, 777)
        assert abs(p[0] - printed) < 3 * math.sqrt(2) * se[0], (name, p, se)


@pytest.mark.parametrize("layout", ["direct", "lds"])
@pytest.mark.parametrize("model", [inputs.STATIC, inputs.DYN_I])
def test_mc_objective_crn_parity(S, ctx, oracle, model, layout):
    """Monte Carlo objective of 70 parameter vectors (two chain tiles, ragged)
    on common paths equals the oracle's prices on the same normals: with the
    path-block sums written straight to device memory (the default here) and
    with blocks of several rounds summed in LDS first (the layout taken when
    the direct partials would not fit; forced by a kernel-layout override)."""
    if layout == "lds":
        ctx = _ctx_with(S, {"SABR_CRN_VARIANT": "9"})
    g = inputs.make_grid([0.25, 0.75], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0, disc=[0.995, 0.985])
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5] if model == inputs.STATIC else [0.2, -0.3, 0.5, 0.4, 0.6]
    tgt, _ = oracle.mc_prices(m, model, xt, 0.7, 1500, 250, 99)
    m.target = tgt
    X = random_params(model, 70, 51)
    f, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(model, 0.7), X,
                                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32,
                                    n_paths=1500, steps_per_year=250, mc_seed=99, want_model=True)
    for i in range(len(X)):
        ref, _ = oracle.mc_prices(m, model, X[i], 0.7, 1500, 250, 99)
        np.testing.assert_allclose(mod[i], ref, rtol=5e-5, atol=1e-7)
        rf = oracle.objective_mc(m, model, X[i], 0.7, 1500, 250, 99)
        assert abs(f[i] - rf) <= 1e-3 * rf + 1e-8


def test_mc_objective_lds_rounds_match_direct(S, ctx, oracle):
    """3000 parameter vectors (47 chain tiles): the LDS layout then takes 87
    path blocks of 18 paths (a full round of 16 and a partial one summed in
    LDS); its prices match the oracle on sampled vectors and the direct
    layout's on all of them."""
    g = inputs.make_grid([0.25, 0.75], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0, disc=[0.995, 0.985])
    m = omkt(oracle, g)
    tgt, _ = oracle.mc_prices(m, inputs.STATIC, [0.2, -0.3, 0.5], 0.7, 1500, 250, 77)
    X = random_params(inputs.STATIC, 3000, 53)
    args = dict(kind=S.SABR_OBJ_MC, precision=S.SABR_FP32, n_paths=1500, steps_per_year=250, mc_seed=77,
                want_model=True)
    mk, pb = S.Market.from_grid(g, target=tgt), S.Problem(inputs.STATIC, 0.7)
    _, mod_direct = S.sabr_objective_batch(ctx, mk, pb, X, **args)
    c = _ctx_with(S, {"SABR_CRN_VARIANT": "9"})
    try:
        _, mod_lds = S.sabr_objective_batch(c, mk, pb, X, **args)
    finally:
        c.close()
    np.testing.assert_allclose(mod_lds, mod_direct, rtol=5e-5, atol=1e-7)
    for i in (0, 1, 63, 64, 1500, 2999):
        ref, _ = oracle.mc_prices(m, inputs.STATIC, X[i], 0.7, 1500, 250, 77)
        np.testing.assert_allclose(mod_lds[i], ref, rtol=5e-5, atol=1e-7)


# --- annealing -----------------------------------------------------------------------------
def smile_request(S, oracle, x_true, noise_sd, prec, n_chains, n_iters, seed, polish=False, noise_seed=1):
    g = inputs.single_smile()
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, x_true, g.meta["beta"])
    if noise_sd:
        tgt = tgt + inputs.vol_noise(noise_seed, len(tgt), noise_sd)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, g.meta["beta"], lb, ub),
                    precision=prec, n_chains=n_chains, n_iters=n_iters, seed=seed, polish=polish)
    return req, m, lb, ub


@pytest.mark.parametrize("n_chains", [64, 600, 1300, 8500, 33000])
def test_sa_fp64_matches_oracle_trajectory(S, ctx, oracle, n_chains):
    """FP64 mode takes the oracle's annealing decisions: same accepted-move
    count and the same best point (600 chains span 3 workgroups, ragged;
    8500 span 67, past the 64 whose level-end slots one wave reads, so one
    workgroup reads them all and hands out the winner; 33000 span 258, read
    by two workgroups whose two results every workgroup compares)."""
    say("sa fp64 chains", n_chains)
    x_true = np.array([0.2, -0.3, 0.5])
    req, m, lb, ub = smile_request(S, oracle, x_true, 1e-4, S.SABR_FP64, n_chains, 200, 0x5AB10001)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, n_chains, 200, 0x5AB10001)
    say("gpu", got["x"], got["f"], got["n_accept"], "oracle", ref["x"], ref["f"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-12)
    assert abs(got["f"] - ref["f"]) <= 1e-12 * ref["f"] + 1e-14 * math.sqrt(ref["f"] * np.sum(m.target ** 2))


def test_sa_single_smile_recovery_fp32_and_fp64(S, ctx, oracle):
    """Single-smile workload (64 chains x 1000): FP64 and FP32 runs and the
    oracle land within 1e-3 of each other; with polish, within 1e-3 of truth
    on noise-free data."""
    x_true = np.array([0.2, -0.3, 0.5])
    r64, m, lb, ub = smile_request(S, oracle, x_true, 1e-4, S.SABR_FP64, 64, 1000, 0x5AB10001)
    r32, _, _, _ = smile_request(S, oracle, x_true, 1e-4, S.SABR_FP32, 64, 1000, 0x5AB10001)
    g64, g32 = S.sabr_calibrate_many(ctx, [r64, r32])
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 64, 1000, 0x5AB10001, cooling=0.99)
    say("fp64", g64["x"], "fp32", g32["x"], "oracle", ref["x"])
    np.testing.assert_allclose(g64["x"], ref["x"], atol=1e-3)
    np.testing.assert_allclose(g32["x"], ref["x"], atol=1e-3)
    p32, _, _, _ = smile_request(S, oracle, x_true, 0.0, S.SABR_FP32, 64, 1000, 7, polish=True)
    gp = S.sabr_calibrate(ctx, p32)
    np.testing.assert_allclose(gp["x"], x_true, atol=1e-3)
    assert gp["f"] <= gp["f_before_polish"] * (1 + 1e-6) + 1e-12


@pytest.mark.parametrize("noise_sd", [0.0, 2e-3])
def test_polish_matches_oracle(S, ctx, oracle, noise_sd):
    """FP64 annealing (the oracle's decisions) followed by the double-precision
    Levenberg-Marquardt polish: GPU and oracle end at the same point."""
    x_true = np.array([0.2, -0.3, 0.5])
    req, m, lb, ub = smile_request(S, oracle, x_true, noise_sd, S.SABR_FP64, 64, 300, 17, polish=True,
                                   noise_seed=9)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 64, 300, 17, polish=True)
    say("polish gpu", got["x"], got["f"], "oracle", ref["x"], ref["f"])
    assert got["f_before_polish"] == pytest.approx(ref["f_before_polish"], rel=1e-12)
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-8)
    assert abs(got["f"] - ref["f"]) <= 1e-9 * ref["f"] + 1e-28
    if noise_sd == 0.0:
        np.testing.assert_allclose(got["x"], x_true, atol=1e-9)


def test_sa_batch_equals_alone(S, ctx, oracle):
    """A request's result does not depend on the other requests of the batch
    (sizes on both sides of the two-lanes-per-chain threshold)."""
    reqs = []
    for k, xt in enumerate(([0.2, -0.3, 0.5], [0.4, 0.2, 1.1], [0.1, -0.7, 0.3], [0.3, 0.1, 0.8])):
        r, _, _, _ = smile_request(S, oracle, np.array(xt), 1e-4, S.SABR_FP32, (256, 320, 1100, 2048)[k], 300,
                                   100 + k)
        reqs.append(r)
    together = S.sabr_calibrate_many(ctx, reqs)
    for r, t in zip(reqs, together):
        alone = S.sabr_calibrate(ctx, r)
        assert np.array_equal(alone["x"], t["x"]) and alone["f"] == t["f"] and alone["n_accept"] == t["n_accept"]


def test_sa_dynamic_case1_fp64_trajectory(S, ctx, oracle):
    g = inputs.make_grid(inputs.dynamic_ladder(6), [np.exp(np.linspace(-0.5, 0.5, 7))] * 6)
    m = omkt(oracle, g)
    xt = [0.2, -0.4, 0.6, 0.3, 0.5]
    tgt = oracle.model_vols(m, oracle.DYN_I, xt, 0.7)
    m.target = tgt
    lb, ub = inputs.box(inputs.DYN_I)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                    precision=S.SABR_FP64, n_chains=64, n_iters=100, seed=5)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.DYN_I, lb, ub, 0.7, 64, 100, 5)
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-12)


def test_sa_mc_objective_trajectory(S, ctx, oracle):
    """Technique II on the device: a tiny Monte Carlo calibration follows the
    oracle's accept decisions (objectives agree to ~1e-6 relative)."""
    g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5]
    tgt, _ = oracle.mc_prices(m, oracle.STATIC, xt, 0.7, 512, 250, 4242)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8,
                    n_iters=20, seed=3, n_paths=512, steps_per_year=250, mc_seed=4242)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 8, 20, 3, weighting=oracle.RELATIVE,
                           objective=oracle.OBJ_MC, mc_paths=512, mc_steps_per_year=250, mc_seed=4242)
    say("mc sa gpu", got, "oracle", ref)
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-12)
    assert abs(got["f"] - ref["f"]) <= 1e-3 * ref["f"]


def _ctx_with(S, env):
    """A context created with lane-layout overrides in the environment."""
    import os
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        return S.sabr_ctx_create(0)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


@pytest.mark.parametrize("model,n_chains,ragged", [(inputs.DYN_I, 2048, False), (inputs.DYN_II, 2048, False),
                                                   (inputs.DYN_I, 300, False), (inputs.DYN_I, 1024, True)])
def test_sa_wide_lane_groups_follow_one_lane_trajectory(S, ctx, oracle, model, n_chains, ragged):
    """Float dynamic requests of many chains spread each chain over up to 16
    lanes (whole rows per lane, the remaining rows split, or a fixed row
    split); only the order of the double partial sums changes, so the accept
    decisions and the result are those of one lane per chain, for every
    schedule (the ragged grid: 13 rows of 5 to 21 strikes, fewer rows than a
    16-lane group)."""
    if ragged:
        T = inputs.dynamic_ladder(20)[:13]
        g = inputs.make_grid(T, [np.exp(np.linspace(-0.5, 0.5, 5 + (3 * i) % 17)) for i in range(13)])
        xt = inputs.dynamic_surface().meta["x_true"]
    elif model == inputs.DYN_I:
        g = inputs.dynamic_surface()
        xt = g.meta["x_true"]
    else:
        g = inputs.make_grid(inputs.dynamic_ladder(10), [np.exp(np.linspace(-0.4, 0.4, 9))] * 10)
        xt = inputs.dynamic_surface().meta["x_true_case2"]
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, model, xt, 0.7)
    lb, ub = inputs.box(model)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(model, 0.7, lb, ub),
                    precision=S.SABR_FP32, n_chains=n_chains, n_iters=60, seed=0x77)
    runs = {}
    for name, env in (("one", {"SABR_LANES_PER_CHAIN": "1"}), ("default", {}),
                      ("16x16", {"SABR_LANES_PER_CHAIN": "16", "SABR_ROW_SPLIT": "16"}),
                      ("8x2", {"SABR_LANES_PER_CHAIN": "8", "SABR_ROW_SPLIT": "2"}),
                      ("16", {"SABR_LANES_PER_CHAIN": "16"}), ("4", {"SABR_LANES_PER_CHAIN": "4"})):
        c = _ctx_with(S, env) if env else ctx
        say("wide lanes", model, name)
        runs[name] = S.sabr_calibrate(c, req)
        if env:
            c.close()
    base = runs["one"]
    for name, r in runs.items():
        say(name, r["x"], r["f"], r["n_accept"])
        assert r["status"] == 0
        assert r["n_accept"] == base["n_accept"], name
        np.testing.assert_allclose(r["x"], base["x"], rtol=0, atol=1e-12)
        assert r["f"] == pytest.approx(base["f"], rel=1e-12)


def test_large_batch_runs_in_resident_parts(S, ctx, oracle):
    """A batch whose workgroups cannot all be resident at once is run as
    consecutive launches; every request still gets its own result."""
    g = inputs.dynamic_surface()
    m = omkt(oracle, g)
    lb, ub = inputs.box(inputs.DYN_I)
    rng = np.random.default_rng(8)
    reqs = []
    for k in range(40):
        xt = lb + (ub - lb) * (0.25 + 0.5 * rng.random(len(lb)))
        tgt = oracle.model_vols(m, inputs.DYN_I, xt, 0.7)
        reqs.append(S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                              precision=S.SABR_FP32, n_chains=1024, n_iters=20, seed=500 + k))
    together = S.sabr_calibrate_many(ctx, reqs)
    assert all(r["status"] == 0 for r in together)
    for i in (0, 21, 39):
        alone = S.sabr_calibrate(ctx, reqs[i])
        assert np.array_equal(alone["x"], together[i]["x"]) and alone["f"] == together[i]["f"]
        assert alone["n_accept"] == together[i]["n_accept"]


def test_caller_workspace_gives_identical_results(S, ctx, oracle):
    """With a caller-owned device workspace the context allocates nothing and
    every result is bit-identical to the library-allocated run; a workspace
    too small for a call is reported as a budget error."""
    import torch
    req, m, lb, ub = smile_request(S, oracle, np.array([0.2, -0.3, 0.5]), 1e-4, S.SABR_FP32, 1100, 200, 31,
                                   polish=True)
    g = inputs.make_grid([0.25, 0.75], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    X = random_params(inputs.STATIC, 50, 4)
    mk = S.Market.from_grid(g, target=np.full(6, 0.2))

    def run(c):
        r = S.sabr_calibrate(c, req)
        f, mod = S.sabr_objective_batch(c, mk, S.Problem(S.SABR_STATIC, 0.7), X, precision=S.SABR_FP32,
                                        want_model=True)
        p, se = S.sabr_mc_price(c, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7, x0=[0.2, -0.3, 0.5]),
                                4096, 250, 9)
        return r, f, mod, p, se

    ref = run(ctx)
    c = S.sabr_ctx_create(0)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    S.sabr_ctx_set_workspace(c, ws)
    for _ in range(2):
        got = run(c)
        assert np.array_equal(got[0]["x"], ref[0]["x"]) and got[0]["f"] == ref[0]["f"]
        for a, b in zip(got[1:], ref[1:]):
            assert np.array_equal(a, b)
    S.sabr_ctx_set_workspace(c, ws, 4096)
    with pytest.raises(S.SabrError) as e:
        S.sabr_calibrate(c, req)
    assert e.value.code == S.SABR_E_BUDGET
    S.sabr_ctx_set_workspace(c, None)
    assert np.array_equal(S.sabr_calibrate(c, req)["x"], ref[0]["x"])
    c.close()


def test_mc_objective_calibration_recovers_truth(S, ctx):
    """Monte Carlo objective calibration with targets priced on the same
    common paths at the true parameters (so the truth is an exact minimum)
    recovers them to 1e-3."""
    g = inputs.make_grid([0.5, 1.0], [np.exp(np.linspace(-0.25, 0.25, 5))] * 2, f0=1.0)
    xt = np.array([0.25, -0.3, 0.45])
    lb, ub = inputs.box(inputs.STATIC)
    _, tgt = S.sabr_objective_batch(ctx, S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7), xt[None, :],
                                    kind=S.SABR_OBJ_MC, precision=S.SABR_FP32, n_paths=2048, steps_per_year=50,
                                    mc_seed=11, want_model=True)
    req = S.Request(S.Market.from_grid(g, target=tgt[0]), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=256,
                    n_iters=150, seed=5, n_paths=2048, steps_per_year=50, mc_seed=11)
    r = S.sabr_calibrate(ctx, req)
    say("mc recovery", r["x"][:3], r["f"])
    assert r["status"] == 0
    np.testing.assert_allclose(r["x"][:3], xt, atol=1e-3)
    assert r["f"] < 1e-6


@pytest.mark.parametrize("n_chains", [64, 1024])
@pytest.mark.parametrize("formula", [0, 1])
@pytest.mark.parametrize("weighting", [0, 1])
def test_sa_float_objective_at_result_matches_oracle(S, ctx, oracle, n_chains, formula, weighting):
    """The annealing kernel's own float objective (one and two lanes per
    chain; ragged rows of 7, 7 and 30 strikes, strikes at and next to the
    forward) at the state it returns, without polish, against the oracle's
    FP64 objective at those parameters, within what a vol error of
    delta = 2e-5 allows (as for the objective batch)."""
    K0 = np.exp(np.linspace(-0.4, 0.5, 7))
    K1 = 1.3 * np.exp(np.array([-1e-2, -1e-4, -1e-7, 0.0, 1e-7, 1e-4, 1e-2]))
    K2 = np.exp(np.linspace(-0.7, 0.6, 30))
    g = inputs.make_grid([0.1, 1.3, 6.0], [K0, K1, K2], f0=1.3)
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.25, -0.4, 0.7], 0.6, False, formula) + 2e-3
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.6, lb, ub),
                    formula=formula, weighting=weighting, precision=S.SABR_FP32, n_chains=n_chains,
                    n_iters=300, chain_len=10, cooling=0.99 ** (1000.0 / 300), seed=0xF10A7 + formula)
    got = S.sabr_calibrate(ctx, req)
    x = np.asarray(got["x"][:3])
    ref_f = oracle.objective_formula(m, oracle.STATIC, x, 0.6, False, formula, weighting)
    ref_v = oracle.model_vols(m, oracle.STATIC, x, 0.6, False, formula)
    w = np.ones_like(tgt) if weighting == 0 else 1.0 / tgt ** 2
    delta = 2e-5
    tol = np.sum((2 * np.abs(tgt - ref_v) * delta + delta ** 2) * w) + 1e-6 * ref_f
    say("float objective at result", n_chains, formula, weighting, got["f"], ref_f, tol)
    assert got["status"] == 0 and np.isfinite(ref_f)
    assert abs(got["f"] - ref_f) <= tol


@pytest.mark.parametrize("prec,n_chains", [(1, 64), (1, 1024), (0, 1024)])
def test_sa_never_accepts_negative_vols(S, ctx, oracle, prec, n_chains):
    """A state whose model vol is not positive has objective +inf (the
    objective's reading of a non-positive vol) and is never accepted.  Ten-year
    maturity with rho near -1 and nu near 2: the Hagan maturity factor of eq.
    "haganf" turns the vol negative everywhere in the box (checked on a grid of
    the box with the oracle), so every chain, in the float hot loop (one and
    two lanes per chain) and in double, rejects every proposal."""
    g = inputs.make_grid([10.0], [[0.7, 1.0, 1.4]], f0=1.0)
    lb, ub = np.array([0.2, -0.99, 1.9]), np.array([0.21, -0.98, 2.0])
    for a in np.linspace(lb[0], ub[0], 4):
        for r in np.linspace(lb[1], ub[1], 4):
            for n in np.linspace(lb[2], ub[2], 4):
                assert max(oracle.sigma_hagan(K, 1.0, 10.0, a, 0.5, r, n) for K in g.K) < 0.0
    tgt = np.full(3, 0.3)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.5, lb, ub),
                    precision=prec, n_chains=n_chains, n_iters=40, chain_len=10, seed=0x5EED)
    got = S.sabr_calibrate(ctx, req)
    say("negative vols", prec, n_chains, got["n_accept"], got["f"])
    assert got["n_accept"] == 0
    assert not np.isfinite(got["f"])
    np.testing.assert_array_equal(got["x"][:3], (lb + ub) / 2)


@pytest.mark.parametrize("n_chains,n_iters,chain_len,n_strikes", [
    (1, 1, 10, 15),      # one chain, one iteration
    (3, 7, 10, 15),      # a single, partial temperature level
    (65, 23, 4, 15),     # two waves of chains, ragged last level
    (300, 40, 10, 1),    # one strike
])
def test_sa_degenerate_sizes_follow_oracle(S, ctx, oracle, n_chains, n_iters, chain_len, n_strikes):
    """Degenerate annealing sizes (one chain, one iteration, a partial last
    level, a one-point grid) take the oracle's decisions in FP64."""
    g = inputs.single_smile() if n_strikes > 1 else inputs.make_grid([1.0], [[1.1]], f0=1.0)
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.2, -0.3, 0.5], 0.7)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    cooling = 0.99 ** (1000.0 / n_iters)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    precision=S.SABR_FP64, n_chains=n_chains, n_iters=n_iters, chain_len=chain_len,
                    cooling=cooling, seed=0x77 + n_chains)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, n_chains, n_iters, 0x77 + n_chains,
                           chain_len=chain_len, cooling=cooling)
    say("degenerate", n_chains, n_iters, chain_len, n_strikes, got["n_accept"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-12)


def test_grid_too_large_for_lds_is_rejected(S, ctx):
    """A grid whose records do not fit the LDS of a workgroup is refused with
    SABR_E_INVAL before anything runs."""
    T = [0.5 + 0.01 * i for i in range(40)]
    g = inputs.make_grid(T, [np.exp(np.linspace(-0.5, 0.5, 100))] * 40, f0=1.0)   # 4000 points
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=np.full(g.n_obs, 0.2)), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    precision=S.SABR_FP64, n_chains=64, n_iters=10)
    with pytest.raises(S.SabrError) as e:
        S.sabr_calibrate(ctx, req)
    assert e.value.code == S.SABR_E_INVAL


def test_polish_grid_too_large_is_rejected_before_annealing(S, ctx):
    """A float grid that fits the annealing kernel but not the double polish
    is refused up front when the polish is requested, and runs without it."""
    T = [0.5 + 0.01 * i for i in range(25)]
    g = inputs.make_grid(T, [np.exp(np.linspace(-0.5, 0.5, 100))] * 25, f0=1.0)   # 2500 points
    lb, ub = inputs.box(inputs.STATIC)
    mk = S.Market.from_grid(g, target=np.full(g.n_obs, 0.2))
    with pytest.raises(S.SabrError) as e:
        S.sabr_calibrate(ctx, S.Request(mk, S.Problem(S.SABR_STATIC, 0.7, lb, ub), precision=S.SABR_FP32,
                                        n_chains=64, n_iters=10, polish=True))
    assert e.value.code == S.SABR_E_INVAL
    r = S.sabr_calibrate(ctx, S.Request(mk, S.Problem(S.SABR_STATIC, 0.7, lb, ub), precision=S.SABR_FP32,
                                        n_chains=64, n_iters=10, polish=False))
    assert r["status"] == 0 and np.isfinite(r["f"])


def test_prepared_batch_repeats_calibrate_bitwise(S, ctx, oracle):
    """A prepared batch (inputs uploaded once) returns, run after run, exactly
    what sabr_calibrate_many returns for the same requests: mixed models,
    precisions and polish, and a group large enough to run in resident parts."""
    g = inputs.dynamic_surface()
    m = omkt(oracle, g)
    lb, ub = inputs.box(inputs.DYN_I)
    rng = np.random.default_rng(12)
    reqs = []
    for k in range(40):
        xt = lb + (ub - lb) * (0.25 + 0.5 * rng.random(len(lb)))
        tgt = oracle.model_vols(m, inputs.DYN_I, xt, 0.7)
        reqs.append(S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                              precision=S.SABR_FP32, n_chains=1024, n_iters=20, seed=700 + k))
    for prec, pol in ((S.SABR_FP32, True), (S.SABR_FP64, False)):
        req, _, _, _ = smile_request(S, oracle, np.array([0.2, -0.3, 0.5]), 1e-4, prec, 512, 300, 41, polish=pol)
        reqs.append(req)
    ref = S.sabr_calibrate_many(ctx, reqs)
    b = S.sabr_batch_prepare(ctx, reqs)
    try:
        for rep in range(2):
            got = S.sabr_batch_run(b)
            for r, (a, e) in enumerate(zip(got, ref)):
                assert a["status"] == 0, (rep, r)
                assert np.array_equal(a["x"], e["x"]) and a["f"] == e["f"], (rep, r)
                assert a["f_before_polish"] == e["f_before_polish"] and a["n_accept"] == e["n_accept"], (rep, r)
                assert a["n_evals"] == e["n_evals"], (rep, r)
            # work of the context between runs leaves the batch unchanged
            S.sabr_calibrate_many(ctx, reqs[-1:])
    finally:
        S.sabr_batch_destroy(b)


def test_prepared_batch_refuses_mc_and_invalid(S, ctx):
    g = inputs.make_grid([0.5], [np.exp(np.linspace(-0.2, 0.2, 5))], f0=1.0)
    lb, ub = inputs.box(inputs.STATIC)
    mc = S.Request(S.Market.from_grid(g, target=np.full(5, 0.05)), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                   kind=S.SABR_OBJ_MC, n_chains=64, n_iters=10, n_paths=1024)
    with pytest.raises(S.SabrError) as e:
        S.sabr_batch_prepare(ctx, [mc])
    assert e.value.code == S.SABR_E_INVAL and "Monte Carlo" in str(e.value)
    bad = S.Request(S.Market.from_grid(g, target=np.full(5, 0.2)), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    n_chains=0, n_iters=10)
    with pytest.raises(S.SabrError) as e:
        S.sabr_batch_prepare(ctx, [bad])
    assert e.value.code == S.SABR_E_INVAL


@pytest.mark.parametrize("n_chains", [2048, 8500])
def test_exchange_wait_bound_reports_timeout(S, ctx, oracle, n_chains):
    """A level-end wait that gives up (forced from the host: a context whose
    bound allows no poll at all) ends every workgroup at once and the call
    returns SABR_E_TIMEOUT; the same request then runs normally (16 and 67
    workgroups: both ways of reading the slots)."""
    req, _, _, _ = smile_request(S, oracle, np.array([0.2, -0.3, 0.5]), 1e-4, S.SABR_FP32, n_chains, 100, 7)
    c = _ctx_with(S, {"SABR_EXCHANGE_SPINS": "0"})
    try:
        with pytest.raises(S.SabrError) as e:
            S.sabr_calibrate(c, req)
        assert e.value.code == S.SABR_E_TIMEOUT
    finally:
        c.close()
    r = S.sabr_calibrate(ctx, req)
    assert r["status"] == 0 and np.isfinite(r["f"])


def _exact_fits(x, beta, T, lb, ub):
    """Exact fits of a noise-free single-maturity Hagan surface: the truth
    and, for beta = 1, the point with the same rho and nu/alpha whose alpha is
    the other positive root of alpha + k alpha^3 = const (k < 0; the oracle
    pin of this invariance is in the oracle tests)."""
    sols = [np.asarray(x, dtype=np.float64)]
    al, rho, nu = (float(v) for v in x)
    c = nu / al
    k = T * (rho * c / 4.0 + (2.0 - 3.0 * rho * rho) * c * c / 24.0)
    if beta == 1.0 and k < 0 and -3.0 * al * al - 4.0 / k > 0:
        a2 = 0.5 * (-al + math.sqrt(-3.0 * al * al - 4.0 / k))
        x2 = np.array([a2, rho, c * a2])
        if np.all(x2 >= lb) and np.all(x2 <= ub):
            sols.append(x2)
    return sols


def test_surface_full_size_sampled(S, ctx, oracle):
    """The benchmark's workload in its launch configuration (24 fits x 4096
    chains x 20000 iterations, float annealing, FP64 polish, one prepared
    batch): on sampled fits, the reported objective equals the oracle's FP64
    objective at the reported parameters, the float objective before the
    polish is no smaller than the polished one (within float accuracy), and
    the noise-free truth, or the other exact fit where beta = 1 allows two
    (fits 20 and 22), is recovered."""
    fits = inputs.surface_fits()
    gens, lb, ub = inputs.surface_true_params(len(fits))
    reqs, truths, mkts = [], [], []
    for k, g in enumerate(fits):
        beta = g.meta["beta"]
        m = omkt(oracle, g)
        while True:
            x = inputs.draw_params(gens[k], lb, ub)
            vol = oracle.model_vols(m, oracle.STATIC, x, beta)
            if np.all(np.isfinite(vol)) and np.all(vol > 0):
                break
        m.target = vol
        reqs.append(S.Request(S.Market.from_grid(g, target=vol), S.Problem(S.SABR_STATIC, beta, lb, ub),
                              precision=S.SABR_FP32, n_chains=4096, n_iters=20000, chain_len=10,
                              cooling=0.99 ** (1000.0 / 20000), seed=0x5AB20000 + k, polish=True))
        truths.append(x)
        mkts.append(m)
    b = S.sabr_batch_prepare(ctx, reqs)
    try:
        res = S.sabr_batch_run(b)
    finally:
        S.sabr_batch_destroy(b)
    for k in (0, 5, 11, 12, 17, 20, 22, 23):
        r, m, beta = res[k], mkts[k], fits[k].meta["beta"]
        ref_f = oracle.objective_formula(m, oracle.STATIC, r["x"], beta)
        say("fit", k, "f", r["f"], "oracle", ref_f, "before polish", r["f_before_polish"])
        assert r["status"] == 0
        assert abs(r["f"] - ref_f) <= 1e-12 * ref_f + 1e-14 * math.sqrt(ref_f * np.sum(m.target ** 2)) + 1e-28
        assert r["f_before_polish"] >= r["f"] - 1e-6 * r["f_before_polish"] - 1e-20
        sols = _exact_fits(truths[k], beta, float(fits[k].T[0]), lb, ub)
        err = min(float(np.max(np.abs(r["x"] - s))) for s in sols)
        say("fit", k, "exact solutions", len(sols), "distance to the nearest", err)
        assert err <= 1e-6


def test_dynamic_full_size_sampled(S, ctx, oracle):
    """The dynamic workload in the benchmark's launch configuration (case I,
    20 x 20 joint fit, 8192 chains x 50000 iterations, float annealing with
    16 lanes per chain, FP64 polish): the reported objective equals the
    oracle's FP64 objective at the reported parameters and the noise-free
    truth is recovered."""
    g = inputs.dynamic_surface()
    xt = g.meta["x_true"]
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.DYN_I, xt, 0.7)
    m.target = tgt
    lb, ub = inputs.box(inputs.DYN_I)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_I, 0.7, lb, ub),
                    precision=S.SABR_FP32, n_chains=8192, n_iters=50000, cooling=0.99 ** (1000.0 / 50000),
                    seed=0x5AB40001, polish=True)
    r = S.sabr_calibrate(ctx, req)
    ref_f = oracle.objective_formula(m, oracle.DYN_I, r["x"], 0.7)
    say("dynamic full size", r["x"], r["f"], "oracle f", ref_f, "before polish", r["f_before_polish"])
    assert r["status"] == 0
    assert abs(r["f"] - ref_f) <= 1e-12 * ref_f + 1e-14 * math.sqrt(ref_f * np.sum(tgt ** 2)) + 1e-28
    np.testing.assert_allclose(r["x"], xt, rtol=0, atol=1e-6)


def test_mc_calibration_full_size_self_consistent(S, ctx, oracle):
    """The Monte Carlo workload in the benchmark's launch configuration (8 x 15
    calls, 1024 chains x 500 iterations x 65536 common paths x 250 steps per
    year) with targets priced on the same paths at the truth: the truth is
    recovered to 1e-3, and the reported objective equals the oracle's Monte
    Carlo objective on the same normals at the reported parameters, within
    what prices at 5e-5 relative allow."""
    g = inputs.mc_grid()
    xt = g.meta["x_true"]
    lb, ub = inputs.box(inputs.STATIC)
    mk = S.Market.from_grid(g)
    _, tgt = S.sabr_objective_batch(ctx, mk, S.Problem(S.SABR_STATIC, 0.7), xt[None, :], kind=S.SABR_OBJ_MC,
                                    precision=S.SABR_FP32, n_paths=65536, steps_per_year=250,
                                    mc_seed=g.meta["mc_seed"], want_model=True)
    req = S.Request(S.Market.from_grid(g, target=tgt[0]), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=1024,
                    n_iters=500, cooling=0.99 ** 2, seed=0x5AB30001, n_paths=65536, steps_per_year=250,
                    mc_seed=g.meta["mc_seed"])
    r = S.sabr_calibrate(ctx, req)
    say("mc full size", r["x"], r["f"])
    assert r["status"] == 0
    np.testing.assert_allclose(r["x"], xt, atol=1e-3)
    # the oracle on all 65536 paths (each FP64 evaluation takes a few seconds)
    m = omkt(oracle, g, target=tgt[0])
    ref_f = oracle.objective_mc(m, oracle.STATIC, r["x"], 0.7, 65536, 250, g.meta["mc_seed"])
    ref_p, _ = oracle.mc_prices(m, oracle.STATIC, r["x"], 0.7, 65536, 250, g.meta["mc_seed"])
    _, got_p = S.sabr_objective_batch(ctx, mk, S.Problem(S.SABR_STATIC, 0.7), r["x"][None, :], kind=S.SABR_OBJ_MC,
                                      precision=S.SABR_FP32, n_paths=65536, steps_per_year=250,
                                      mc_seed=g.meta["mc_seed"], want_model=True)
    np.testing.assert_allclose(got_p[0], ref_p, rtol=5e-5, atol=1e-7)
    # relative price residuals e_j agree to delta = 5e-5, so |df| <= sum (2 |e_j| delta + delta^2)
    delta, n = 5e-5, g.n_obs
    tol = 2.0 * math.sqrt(ref_f * n) * delta + n * delta ** 2 + 1e-3 * ref_f
    say("oracle f", ref_f, "tol", tol)
    assert abs(r["f"] - ref_f) <= tol
