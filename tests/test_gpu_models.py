"""GPU parity of the case II constraint, beta-free annealing, the
at-the-money start point and the cliquet, through the C ABI, against the
FP64 oracle on the same seeded inputs.

Tolerances:
  case II model vols, FP64   : 1e-10 relative (device: composite 8-point
                               Gauss-Legendre; oracle: adaptive quadrature);
  case II objective, FP64    : |df| <= 2e-10 sqrt(f sum v^2) + 1e-12 f (what that
                               vol accuracy allows);
  model vols, FP32           : 2e-5 absolute vol;
  FP64 annealing             : the oracle's decisions (same accepted-move
                               count, x within 1e-12);
  Monte Carlo prices, FP32   : 5e-5 relative on identical normals (+1e-7 abs);
  cliquet, FP32 / FP64       : 1e-4 / 1e-9 relative on identical normals;
  antithetic standard errors : FP64 1e-6 relative, FP32 2e-3 relative (pair means
                               of float payoffs);
  at-the-money start point   : 1e-13 relative (device log/pow against glibc).
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


def case2_margin(x, t_max, n=200001):
    """Distance of rho(t), nu(t) from the constraint bounds on (0, t_max] by
    dense sampling (positive: feasible), used only to skip vectors within
    rounding of the boundary."""
    t = np.linspace(1e-12, t_max, n)
    rho = (x[1] + x[7] * t) * np.exp(-x[3] * t) + x[5]
    nu = (x[2] + x[8] * t) * np.exp(-x[4] * t) + x[6]
    return min(1 - rho.max(), rho.min() + 1, nu.min())


# Vectors on both sides of the constraint, including growing exponentials
# (negative rates) whose interior extremum leaves the bounds (t_max = 3).
CASE2_EDGE = [
    [0.2, -0.9, 0.6, -0.5, 0.3, -0.05, 0.0, 0.3, 0.0],    # interior min of rho below -1
    [0.2, -0.9, 0.6, -0.5, 0.3, 0.2, 0.0, 0.3, 0.0],      # the same lifted: feasible? decided below
    [0.2, 0.9, 0.6, -0.5, 0.3, 0.05, 0.0, -0.3, 0.0],     # interior max of rho above 1
    [0.2, 0.0, -0.6, 0.0, -0.4, 0.0, 0.605, 0.0, 0.2],    # nu dips below 0 inside
    [0.2, 0.95, 0.5, 1.0, 1.0, 0.1, 0.0, 0.0, 0.0],       # rho(0) = 1.05
    [0.2, -0.3, 0.5, 0.3, 0.5, 0.1, -0.05, 0.2, 0.3],     # the dynamic workload's case II truth
]


def case2_vectors(n, seed):
    rng = np.random.default_rng(seed)
    lb = np.array([0.05, -0.95, 0.05, -0.6, -0.6, -0.5, -0.5, -1.0, -1.0])
    ub = np.array([0.8, 0.95, 1.5, 3.0, 3.0, 0.5, 0.5, 1.0, 1.0])
    X = lb + (ub - lb) * rng.random((n, 9))
    return np.vstack([np.array(CASE2_EDGE), X])


@pytest.mark.parametrize("prec", [0, 1])
def test_case2_objective_rejects_exactly_the_infeasible_vectors(S, ctx, oracle, prec):
    """Section 5: case II vectors outside rho(t) in [-1, 1], nu(t) > 0 on
    (0, T_max] are rejected (objective +inf) exactly where the oracle's
    constraint check fails, growing exponentials included; the feasible ones
    match the oracle's objective and vols."""
    g = inputs.make_grid([0.25, 1.0, 3.0], [np.exp(np.linspace(-0.4, 0.4, 5))] * 3)
    m = omkt(oracle, g)
    xt = np.array(CASE2_EDGE[-1])
    tgt = oracle.model_vols(m, oracle.DYN_II, xt, 0.7)
    m.target = tgt
    X = case2_vectors(200, 314)
    f, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_II, 0.7), X,
                                    precision=prec, want_model=True)
    n_feas = n_infeas = 0
    for i in range(len(X)):
        feas = oracle.case2_feasible(X[i], 3.0)
        if abs(case2_margin(X[i], 3.0)) < 1e-7:
            continue
        if not feas:
            n_infeas += 1
            assert f[i] == np.inf, (i, X[i], f[i])
            continue
        n_feas += 1
        ref_v = oracle.model_vols(m, oracle.DYN_II, X[i], 0.7)
        ok = np.isfinite(ref_v) & (ref_v > 0) & (ref_v < 5)
        if prec == S.SABR_FP64:
            np.testing.assert_allclose(mod[i][ok], ref_v[ok], rtol=1e-10)
            ref_f = oracle.objective_formula(m, oracle.DYN_II, X[i], 0.7)
            if np.isfinite(ref_f):
                tol = 2e-10 * math.sqrt(ref_f * np.sum(ref_v ** 2)) + 1e-12 * ref_f + 1e-28
                assert abs(f[i] - ref_f) <= tol, (i, f[i], ref_f)
            else:
                assert f[i] == np.inf
        else:
            assert np.max(np.abs(mod[i][ok] - ref_v[ok])) < 2e-5
    say("case II vectors: feasible", n_feas, "infeasible", n_infeas)
    assert n_feas > 20 and n_infeas > 20


def case2_problem(S, oracle):
    g = inputs.make_grid([0.25, 1.0, 2.0], [np.exp(np.linspace(-0.4, 0.4, 5))] * 3)
    m = omkt(oracle, g)
    xt = inputs.dynamic_surface().meta["x_true_case2"]
    tgt = oracle.model_vols(m, oracle.DYN_II, xt, 0.7)
    m.target = tgt
    lb, ub = inputs.box(inputs.DYN_II)
    return g, m, tgt, lb, ub


def test_case2_fp64_annealing_follows_oracle(S, ctx, oracle):
    """Case II annealing in FP64 (Section 5, Technique I): every proposal
    that leaves the constraints is rejected on both sides, and the device
    takes the oracle's decisions (same accepted-move count and end point)."""
    g, m, tgt, lb, ub = case2_problem(S, oracle)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_II, 0.7, lb, ub),
                    precision=S.SABR_FP64, n_chains=64, n_iters=60, seed=0x2C2)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.DYN_II, lb, ub, 0.7, 64, 60, 0x2C2)
    say("case II gpu", got["x"], got["n_accept"], "oracle", ref["x"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-12)
    assert oracle.case2_feasible(got["x"], 2.0)


def test_case2_infeasible_start_point_is_refused(S, ctx, oracle):
    """A case II start point outside the constraints (rho(0) = 1.1) is
    refused with SABR_E_INFEASIBLE by the formula and the Monte Carlo
    calibrations, and its objective is +inf."""
    g, m, tgt, lb, ub = case2_problem(S, oracle)
    x0 = 0.5 * (lb + ub)
    x0[1], x0[5] = 0.9, 0.2
    assert not oracle.case2_feasible(x0, 2.0)
    for kind in (S.SABR_OBJ_FORMULA, S.SABR_OBJ_MC):
        for prec in (S.SABR_FP64, S.SABR_FP32):
            t = tgt if kind == S.SABR_OBJ_FORMULA else np.full(len(tgt), 0.05)
            req = S.Request(S.Market.from_grid(g, target=t), S.Problem(S.SABR_DYN_II, 0.7, lb, ub, x0=x0),
                            kind=kind, precision=prec, n_chains=8, n_iters=10, seed=3, n_paths=256,
                            weighting=S.SABR_W_RELATIVE if kind == S.SABR_OBJ_MC else S.SABR_W_ABSOLUTE)
            with pytest.raises(S.SabrError) as e:
                S.sabr_calibrate(ctx, req)
            assert e.value.code == S.SABR_E_INFEASIBLE, (kind, prec)
    f, _ = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_II, 0.7),
                                  x0[None, :], precision=S.SABR_FP64)
    assert f[0] == np.inf


def test_case2_mc_objective_crn_parity(S, ctx, oracle):
    """Technique II for case II (eq. "el_fun_3" inside the scheme of eq.
    "dis_SABRd"): Monte Carlo prices of 70 parameter vectors on common paths
    equal the oracle's on the same normals; infeasible vectors give +inf."""
    g = inputs.make_grid([0.25, 0.75], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0, disc=[0.995, 0.985])
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5, 0.4, 0.6, 0.05, -0.05, 0.1, 0.2]
    tgt, _ = oracle.mc_prices(m, oracle.DYN_II, xt, 0.7, 1500, 250, 99)
    m.target = tgt
    rng = np.random.default_rng(52)
    lb, ub = inputs.box(inputs.DYN_II)
    lb, ub = lb.copy(), ub.copy()
    lb[5:9] *= 0.3
    ub[5:9] *= 0.3
    X = lb + (ub - lb) * rng.random((70, 9))
    X[:3] = [xt, CASE2_EDGE[4], CASE2_EDGE[0]]
    f, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_II, 0.7), X,
                                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32,
                                    n_paths=1500, steps_per_year=250, mc_seed=99, want_model=True)
    n_inf = 0
    for i in range(len(X)):
        if not oracle.case2_feasible(X[i], 0.75):
            assert f[i] == np.inf
            n_inf += 1
            continue
        ref, _ = oracle.mc_prices(m, oracle.DYN_II, X[i], 0.7, 1500, 250, 99)
        np.testing.assert_allclose(mod[i], ref, rtol=5e-5, atol=1e-7)
        rf = oracle.objective_mc(m, oracle.DYN_II, X[i], 0.7, 1500, 250, 99)
        assert abs(f[i] - rf) <= 1e-3 * rf + 1e-8
    say("case II MC: infeasible", n_inf)
    assert n_inf >= 2 and f[0] < 1e-7


def test_case2_mc_annealing_follows_oracle(S, ctx, oracle):
    """A tiny case II Technique II calibration (8 chains x 20 iterations x
    512 common paths) takes the oracle's accept decisions."""
    g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5, 0.4, 0.6, 0.05, -0.05, 0.1, 0.2]
    tgt, _ = oracle.mc_prices(m, oracle.DYN_II, xt, 0.7, 512, 250, 4243)
    m.target = tgt
    lb, ub = inputs.box(inputs.DYN_II)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_DYN_II, 0.7, lb, ub),
                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8,
                    n_iters=20, seed=13, n_paths=512, steps_per_year=250, mc_seed=4243)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.DYN_II, lb, ub, 0.7, 8, 20, 13, weighting=oracle.RELATIVE,
                           objective=oracle.OBJ_MC, mc_paths=512, mc_steps_per_year=250, mc_seed=4243)
    say("case II mc sa gpu", got["x"], got["n_accept"], "oracle", ref["x"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-12)
    assert abs(got["f"] - ref["f"]) <= 1e-3 * ref["f"]


# --- beta calibrated (Section 3) -------------------------------------------------------
@pytest.mark.parametrize("model", [inputs.STATIC, inputs.DYN_I])
def test_beta_free_fp64_annealing_follows_oracle(S, ctx, oracle, model):
    """With beta among the calibrated parameters (its own coordinate in the
    box [0, 1]) the FP64 annealing takes the oracle's decisions."""
    if model == inputs.STATIC:
        g = inputs.make_grid([0.5, 2.0], [np.exp(np.linspace(-0.5, 0.5, 9))] * 2, f0=1.0)
        g.fwd = np.array([0.9, 1.3])
        xt = [0.25, -0.3, 0.5, 0.6]
    else:
        g = inputs.make_grid(inputs.dynamic_ladder(6), [np.exp(np.linspace(-0.5, 0.5, 7))] * 6)
        xt = [0.2, -0.4, 0.6, 0.3, 0.5, 0.6]
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, model, xt, 0.0, beta_free=True)
    m.target = tgt
    lb, ub = inputs.box(model, beta_free=True)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(model, 0.0, lb, ub, beta_free=True),
                    precision=S.SABR_FP64, n_chains=64, n_iters=120, seed=0xBF + model)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, model, lb, ub, 0.0, 64, 120, 0xBF + model, beta_free=True)
    say("beta free", model, got["x"], got["n_accept"], "oracle", ref["x"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], rtol=0, atol=1e-12)


def test_beta_free_fp32_recovers_truth_with_polish(S, ctx, oracle):
    """Float annealing with beta calibrated, then the FP64 polish, on a
    noise-free surface of four forwards: every parameter, beta included,
    within 1e-3 of the truth."""
    T = [0.25, 0.5, 1.0, 2.0]
    g = inputs.make_grid(T, [np.exp(np.linspace(-0.4, 0.4, 9))] * 4, f0=1.0)
    g.fwd = np.array([0.8, 1.0, 1.25, 1.6])
    xt = np.array([0.25, -0.3, 0.5, 0.6])
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, xt, 0.0, beta_free=True)
    lb, ub = inputs.box(inputs.STATIC, beta_free=True)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.0, lb, ub, beta_free=True),
                    precision=S.SABR_FP32, n_chains=1024, n_iters=2000, seed=0xBF32, polish=True)
    got = S.sabr_calibrate(ctx, req)
    say("beta free fp32", got["x"], got["f"])
    np.testing.assert_allclose(got["x"], xt, atol=1e-3)


# --- at-the-money start point (Section 3) ---------------------------------------------
def atm_grid():
    T = [0.08, 0.5, 1.0, 2.0, 5.0]
    rows = [np.exp(np.linspace(-0.3, 0.3, 7)) * f for f in (0.9, 1.05, 1.2, 1.5, 2.1)]
    rows[2] = rows[2][[0, 1, 2, 4, 5, 6]]      # no strike at the forward: interpolated
    g = inputs.make_grid(T, rows)
    g.fwd = np.array([0.9, 1.05, 1.2, 1.5, 2.1])
    return g


@pytest.mark.parametrize("model,beta_free", [(inputs.STATIC, False), (inputs.STATIC, True), (inputs.DYN_I, True),
                                             (inputs.DYN_II, False)])
def test_atm_seed_matches_oracle(S, ctx, oracle, model, beta_free):
    g = atm_grid()
    m = omkt(oracle, g)
    xt = {inputs.STATIC: [0.3, -0.2, 0.4], inputs.DYN_I: [0.3, -0.2, 0.4, 0.3, 0.5],
          inputs.DYN_II: [0.3, -0.2, 0.4, 0.3, 0.5, 0.05, 0.05, 0.1, 0.1]}[model]
    xt = list(xt) + ([0.65] if beta_free else [])
    tgt = oracle.model_vols(m, model, xt, 0.65, beta_free=beta_free)
    m.target = tgt
    lb, ub = inputs.box(model, beta_free)
    got = S.sabr_atm_seed(ctx, S.Market.from_grid(g, target=tgt), S.Problem(model, 0.65, lb, ub,
                                                                            beta_free=beta_free))
    ref = oracle.atm_seed(m, model, lb, ub, 0.65, beta_free=beta_free)
    say("atm seed", model, beta_free, got, ref)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)
    if beta_free:
        assert abs(got[-1] - 0.65) < 0.1         # the log-log slope sees beta through the T-correction


def test_atm_seeded_calibration_follows_oracle(S, ctx, oracle):
    """A calibration started from the at-the-money seed (passed back as x0)
    takes the oracle's decisions from the oracle's own seed."""
    g = inputs.single_smile()
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.2, -0.3, 0.5], 0.7)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    x0 = S.sabr_atm_seed(ctx, S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub))
    x0_ref = oracle.atm_seed(m, oracle.STATIC, lb, ub, 0.7)
    np.testing.assert_allclose(x0, x0_ref, rtol=1e-14)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub, x0=x0_ref),
                    precision=S.SABR_FP64, n_chains=64, n_iters=200, seed=0xA7)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, oracle.STATIC, lb, ub, 0.7, 64, 200, 0xA7, x0=x0_ref)
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-12)


def test_atm_seed_rejects_bad_grids(S, ctx):
    g = inputs.make_grid([0.5], [[1.1, 0.9, 1.0]])
    lb, ub = inputs.box(inputs.STATIC)
    with pytest.raises(S.SabrError) as e:
        S.sabr_atm_seed(ctx, S.Market.from_grid(g, target=np.full(3, 0.2)), S.Problem(S.SABR_STATIC, 0.7, lb, ub))
    assert e.value.code == S.SABR_E_INVAL
    g = inputs.make_grid([0.5], [[0.9, 1.0, 1.1]])
    with pytest.raises(S.SabrError) as e:
        S.sabr_atm_seed(ctx, S.Market.from_grid(g, target=np.array([0.2, 0.0, 0.2])),
                        S.Problem(S.SABR_STATIC, 0.7, lb, ub))
    assert e.value.code == S.SABR_E_INVAL


# --- cliquet (Section 6) --------------------------------------------------------------------
CLIQUET = dict(reset_T=[0.25, 0.5, 0.75, 1.0], local_floor=-0.02, local_cap=0.02, global_floor=0.0,
               global_cap=0.2)


@pytest.mark.parametrize("model,x,beta", [
    (inputs.STATIC, [0.3, -0.5, 0.8], 0.7),
    (inputs.DYN_I, [0.393329, -1.0, 0.941565, 0.001, 1.246906], 1.0),
    (inputs.DYN_II, [0.398436, -0.964678, 1.285129, 0.0, 2.059560, 0.101632, -0.086294, 0.0, 1.302296], 0.999579),
])
@pytest.mark.parametrize("prec", [1, 0])
def test_cliquet_matches_oracle_on_identical_normals(S, ctx, oracle, model, x, beta, prec):
    """The paper's cliquet (D = 4 quarterly resets, local limits +-2 %,
    global [0, 0.2]) on 3000 paths (a ragged last tile) of the three models."""
    kw = dict(CLIQUET)
    ref, rse = oracle.mc_cliquet(model, x, beta, 1.3, kw["reset_T"], kw["local_floor"], kw["local_cap"],
                                 kw["global_floor"], kw["global_cap"], 3000, 250, 0xC11, disc=0.97)
    got, gse = S.sabr_mc_cliquet(ctx, S.Problem(model, beta, x0=x), 1.3, kw["reset_T"], kw["local_floor"],
                                 kw["local_cap"], kw["global_floor"], kw["global_cap"], 3000, 250, 0xC11,
                                 disc=0.97, precision=prec)
    say("cliquet", model, prec, got, ref)
    assert 0.0 < ref < 0.06 * 0.97
    if prec == S.SABR_FP32:
        assert got == pytest.approx(ref, rel=1e-4)
    else:
        assert got == pytest.approx(ref, rel=1e-9)
        assert gse == pytest.approx(rse, rel=1e-6)


def test_cliquet_limits_and_validation(S, ctx, oracle):
    """Equal floor and cap give that value exactly; reset dates on the same
    step, fewer than two dates and a floor above its cap are refused."""
    p = S.Problem(S.SABR_STATIC, 0.7, x0=[0.3, -0.5, 0.8])
    v, se = S.sabr_mc_cliquet(ctx, p, 1.0, [0.25, 0.5], -1.0, 1.0, 0.03, 0.03, 1000, 250, 1, disc=0.9,
                              precision=S.SABR_FP64)
    assert v == pytest.approx(0.9 * 0.03, rel=1e-14) and se < 1e-9
    for bad in (dict(reset_T=[0.25, 0.2501]), dict(reset_T=[0.25]), dict(local_floor=0.1)):
        kw = dict(CLIQUET)
        kw.update(bad)
        with pytest.raises(S.SabrError) as e:
            S.sabr_mc_cliquet(ctx, p, 1.0, kw["reset_T"], kw["local_floor"], kw["local_cap"], kw["global_floor"],
                              kw["global_cap"], 1000, 250, 1)
        assert e.value.code == S.SABR_E_INVAL


# --- nu = 0 in the float hot loop (Section 2.1: z / x(z) -> 1) ---------------------------
def test_fp32_objective_at_zero_nu_matches_oracle(S, ctx, oracle):
    """nu = 0 (allowed by the box) has the finite limit z / x(z) = 1; the float
    objective with and without model output and the oracle agree."""
    g = inputs.make_grid([0.1, 1.3, 6.0], [np.exp(np.linspace(-0.4, 0.5, 7))] * 3, f0=1.3)
    m = omkt(oracle, g)
    tgt = oracle.model_vols(m, oracle.STATIC, [0.25, -0.4, 0.7], 0.6) + 2e-3
    m.target = tgt
    X = np.array([[0.25, -0.4, 0.0], [0.3, 0.2, 0.0], [0.25, -0.4, 1e-30], [0.25, -0.4, 0.7]])
    mk, pb = S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.6)
    f0, _ = S.sabr_objective_batch(ctx, mk, pb, X, precision=S.SABR_FP32)
    f1, mod = S.sabr_objective_batch(ctx, mk, pb, X, precision=S.SABR_FP32, want_model=True)
    for i in range(len(X)):
        ref_f = oracle.objective_formula(m, oracle.STATIC, X[i], 0.6)
        ref_v = oracle.model_vols(m, oracle.STATIC, X[i], 0.6)
        tol = np.sum(2 * np.abs(tgt - ref_v) * 2e-5 + 4e-10) + 1e-6 * ref_f
        say("nu", X[i][2], f0[i], f1[i], ref_f)
        assert np.isfinite(f0[i]) and abs(f0[i] - ref_f) <= tol and abs(f1[i] - ref_f) <= tol
        assert np.max(np.abs(mod[i] - ref_v)) < 2e-5


# Antithetic path pairs (a variance reduction the paper does not use): the
# same parity bars as the plain scheme, on the oracle's pairs.
ANTI_CASES = [
    (inputs.STATIC, [0.3, -0.5, 0.8], 0.7),
    (inputs.DYN_I, [0.393329, -1.0, 0.941565, 0.001, 1.246906], 1.0),
    (inputs.DYN_II, [0.398436, -0.964678, 1.285129, 0.0, 2.059560, 0.101632, -0.086294, 0.0, 1.302296], 0.999579),
]


@pytest.mark.parametrize("model,x,beta", ANTI_CASES)
@pytest.mark.parametrize("prec", [1, 0])
def test_mc_price_antithetic_matches_oracle(S, ctx, oracle, model, x, beta, prec):
    """European calls on 3000 paths (1500 pairs; a ragged last tile) under the
    antithetic scheme: prices and pair-based standard errors equal the
    oracle's on the same pairs of normals; the entry point without
    allocation gives the same bits."""
    say("mc antithetic", model, prec)
    g = inputs.make_grid([0.25, 0.5, 1.0], [np.exp(np.linspace(-0.3, 0.3, 5))] * 3, f0=1.0,
                         disc=[0.99, 0.98, 0.96])
    m = omkt(oracle, g)
    ref, rse = oracle.mc_prices(m, model, x, beta, 3000, 250, 0xA17, scheme=oracle.MC_ANTITHETIC)
    mk, pb = S.Market.from_grid(g), S.Problem(model, beta, x0=x)
    got, gse = S.sabr_mc_price(ctx, mk, pb, 3000, 250, 0xA17, precision=prec, scheme=S.SABR_MC_ANTITHETIC)
    if prec == S.SABR_FP32:
        np.testing.assert_allclose(got, ref, rtol=5e-5, atol=1e-7)
        np.testing.assert_allclose(gse, rse, rtol=2e-3, atol=1e-8)
    else:
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-13)
        np.testing.assert_allclose(gse, rse, rtol=1e-6)
    na, nse = S.sabr_mc_price_noalloc(ctx, mk, pb, 3000, 250, 0xA17, precision=prec, scheme=S.SABR_MC_ANTITHETIC)
    assert np.array_equal(na, got) and np.array_equal(nse, gse)
    # the pairs differ from the plain paths: the plain estimate is another one
    plain, _ = S.sabr_mc_price(ctx, mk, pb, 3000, 250, 0xA17, precision=prec)
    assert not np.array_equal(plain, got)


@pytest.mark.parametrize("model", [inputs.STATIC, inputs.DYN_I])
def test_mc_objective_antithetic_matches_oracle(S, ctx, oracle, model):
    """Monte Carlo objective of 70 parameter vectors on common antithetic
    pairs (1500 paths): model prices and relative-error objective equal the
    oracle's on the same pairs."""
    g = inputs.make_grid([0.25, 0.75], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0, disc=[0.995, 0.985])
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5] if model == inputs.STATIC else [0.2, -0.3, 0.5, 0.4, 0.6]
    tgt, _ = oracle.mc_prices(m, model, xt, 0.7, 1500, 250, 98, scheme=oracle.MC_ANTITHETIC)
    m.target = tgt
    lb, ub = inputs.box(model)
    rng = np.random.default_rng(52)
    X = lb + (ub - lb) * (0.2 + 0.6 * rng.random((70, len(lb))))
    f, mod = S.sabr_objective_batch(ctx, S.Market.from_grid(g, target=tgt), S.Problem(model, 0.7), X,
                                    kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32,
                                    n_paths=1500, steps_per_year=250, mc_seed=98, want_model=True,
                                    mc_scheme=S.SABR_MC_ANTITHETIC)
    for i in range(0, len(X), 7):
        ref, _ = oracle.mc_prices(m, model, X[i], 0.7, 1500, 250, 98, scheme=oracle.MC_ANTITHETIC)
        np.testing.assert_allclose(mod[i], ref, rtol=5e-5, atol=1e-7)
        rf = oracle.objective_mc(m, model, X[i], 0.7, 1500, 250, 98, scheme=oracle.MC_ANTITHETIC)
        assert abs(f[i] - rf) <= 1e-3 * rf + 1e-8


def test_mc_calibration_antithetic_follows_oracle(S, ctx, oracle):
    """Technique II on antithetic pairs: a tiny Monte Carlo calibration (8
    chains x 20 iterations, 512 paths) takes the oracle's accept decisions on
    the same pairs (objectives agree to ~1e-6 relative)."""
    g = inputs.make_grid([0.25, 0.5], [np.exp(np.linspace(-0.2, 0.2, 3))] * 2, f0=1.0)
    m = omkt(oracle, g)
    xt = [0.2, -0.3, 0.5]
    tgt, _ = oracle.mc_prices(m, inputs.STATIC, xt, 0.7, 512, 250, 4243, scheme=oracle.MC_ANTITHETIC)
    m.target = tgt
    lb, ub = inputs.box(inputs.STATIC)
    req = S.Request(S.Market.from_grid(g, target=tgt), S.Problem(S.SABR_STATIC, 0.7, lb, ub), kind=S.SABR_OBJ_MC,
                    weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=8, n_iters=20, seed=3,
                    n_paths=512, steps_per_year=250, mc_seed=4243, mc_scheme=S.SABR_MC_ANTITHETIC)
    got = S.sabr_calibrate(ctx, req)
    ref = oracle.calibrate(m, inputs.STATIC, lb, ub, 0.7, 8, 20, 3, objective=oracle.OBJ_MC,
                           weighting=oracle.RELATIVE, mc_paths=512, mc_steps_per_year=250, mc_seed=4243,
                           mc_scheme=oracle.MC_ANTITHETIC)
    say("mc anti calibration", got["x"], got["n_accept"], ref["x"], ref["n_accept"])
    assert got["n_accept"] == ref["n_accept"]
    np.testing.assert_allclose(got["x"], ref["x"], atol=1e-12)
    assert abs(got["f"] - ref["f"]) <= 1e-3 * ref["f"]


@pytest.mark.parametrize("prec", [1, 0])
def test_cliquet_antithetic_matches_oracle(S, ctx, oracle, prec):
    """The paper's cliquet on 3000 antithetic paths: price and pair-based
    standard error equal the oracle's on the same pairs."""
    kw = dict(CLIQUET)
    model, x, beta = ANTI_CASES[1]
    ref, rse = oracle.mc_cliquet(model, x, beta, 1.3, kw["reset_T"], kw["local_floor"], kw["local_cap"],
                                 kw["global_floor"], kw["global_cap"], 3000, 250, 0xC12, disc=0.97,
                                 scheme=oracle.MC_ANTITHETIC)
    got, gse = S.sabr_mc_cliquet(ctx, S.Problem(model, beta, x0=x), 1.3, kw["reset_T"], kw["local_floor"],
                                 kw["local_cap"], kw["global_floor"], kw["global_cap"], 3000, 250, 0xC12,
                                 disc=0.97, precision=prec, scheme=S.SABR_MC_ANTITHETIC)
    if prec == S.SABR_FP32:
        assert got == pytest.approx(ref, rel=1e-4)
    else:
        assert got == pytest.approx(ref, rel=1e-9)
        assert gse == pytest.approx(rse, rel=1e-6)


def test_antithetic_validation(S, ctx):
    """An odd path count or an unknown scheme is refused; the serving loop
    takes the plain scheme only."""
    g = inputs.make_grid([0.5], [np.exp(np.linspace(-0.2, 0.2, 4))], f0=1.0)
    mk, pb = S.Market.from_grid(g), S.Problem(S.SABR_STATIC, 0.7, x0=[0.2, -0.3, 0.5])
    for n, sch in ((1001, S.SABR_MC_ANTITHETIC), (1000, 2)):
        with pytest.raises(S.SabrError) as e:
            S.sabr_mc_price(ctx, mk, pb, n, 250, 1, scheme=sch)
        assert e.value.code == S.SABR_E_INVAL
    lb, ub = inputs.box(inputs.STATIC)
    srv = S.Server(ctx, max_slots=4)
    try:
        req = S.Request(S.Market.from_grid(g, target=np.full(4, 0.05)), S.Problem(S.SABR_STATIC, 0.7, lb, ub),
                        kind=S.SABR_OBJ_MC, weighting=S.SABR_W_RELATIVE, precision=S.SABR_FP32, n_chains=16,
                        n_iters=10, n_paths=1024, mc_scheme=S.SABR_MC_ANTITHETIC)
        with pytest.raises(S.SabrError) as e:
            srv.submit(req)
        assert e.value.code == S.SABR_E_INVAL and "plain" in str(e.value)
    finally:
        srv.close()
