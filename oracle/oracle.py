"""ctypes binding of the FP64 oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the product library.  The
oracle shares no code with the HIP path; see sabr_oracle.c for what each
function follows in the paper.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "sabr_oracle.c")

STATIC, DYN_I, DYN_II = 0, 1, 2
HAGAN, OBLOJ, EXPANSION = 0, 1, 2
ABSOLUTE, RELATIVE = 0, 1
OBJ_FORMULA, OBJ_MC = 0, 1
MC_PLAIN, MC_ANTITHETIC = 0, 1


def build(force=False):
    """Compile liboracle.so with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None
_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)
_I64 = C.POINTER(C.c_int64)
_U32 = C.POINTER(C.c_uint32)


class SAProblem(C.Structure):
    _fields_ = [("model", C.c_int32), ("formula", C.c_int32), ("weighting", C.c_int32),
                ("objective", C.c_int32), ("beta", C.c_double), ("beta_free", C.c_int32),
                ("n_par", C.c_int32), ("lb", _D), ("ub", _D), ("x0", _D), ("n_mat", C.c_int32),
                ("T", _D), ("fwd", _D), ("disc", _D), ("offs", _I32), ("K", _D), ("target", _D),
                ("n_chains", C.c_int32), ("n_iters", C.c_int32), ("chain_len", C.c_int32),
                ("T0", C.c_double), ("cooling", C.c_double), ("step0", C.c_double),
                ("step_min", C.c_double), ("seed", C.c_uint64), ("polish", C.c_int32),
                ("mc_paths", C.c_int64), ("mc_steps_per_year", C.c_int32), ("mc_scheme", C.c_int32),
                ("mc_seed", C.c_uint64)]


class SAResult(C.Structure):
    _fields_ = [("x", C.c_double * 10), ("f", C.c_double), ("f_before_polish", C.c_double),
                ("n_evals", C.c_int64), ("n_accept", C.c_int64), ("status", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        L.or_philox4x32_10.argtypes = [_U32, _U32, _U32]
        L.or_mc_normals.argtypes = [C.c_uint64, C.c_int64, C.c_int32, _D, _D]
        L.or_path_normals.argtypes = [C.c_uint64, C.c_int, C.c_int64, C.c_int32, _D, _D]
        for name in ("or_sigma_hagan", "or_sigma_obloj", "or_sigma_expansion"):
            getattr(L, name).argtypes = [C.c_double] * 7
            getattr(L, name).restype = C.c_double
        L.or_z_over_x.argtypes = [C.c_double, C.c_double]
        L.or_z_over_x.restype = C.c_double
        L.or_case1_integrals.argtypes = [C.c_double] * 5 + [_D]
        L.or_case2_integrals.argtypes = [C.c_double, _D, _D]
        L.or_quad_integrals.argtypes = [C.c_int, C.c_double, _D, _D]
        L.or_sigma_dyn.argtypes = [C.c_double] * 5 + [_D]
        L.or_sigma_dyn.restype = C.c_double
        L.or_black_call.argtypes = [C.c_double] * 5
        L.or_black_call.restype = C.c_double
        L.or_model_vols.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, _D, C.c_int,
                                    _D, _D, _I32, _D, _D]
        L.or_objective_formula.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                           _D, C.c_int, _D, _D, _I32, _D, _D]
        L.or_objective_formula.restype = C.c_double
        L.or_mc_prices.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _D, C.c_int, _D, _D, _D,
                                   _I32, _D, C.c_int64, C.c_int32, C.c_uint64, C.c_int, _D, _D]
        L.or_objective_mc.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, _D, C.c_int,
                                      _D, _D, _D, _I32, _D, _D, C.c_int64, C.c_int32, C.c_uint64, C.c_int]
        L.or_objective_mc.restype = C.c_double
        L.or_case2_feasible.argtypes = [_D, C.c_double]
        L.or_mc_cliquet.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _D, C.c_double, C.c_double, C.c_int,
                                    _D, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int32,
                                    C.c_uint64, C.c_int, _D, _D]
        L.or_atm_vol.argtypes = [C.c_int, _D, _D, C.c_double]
        L.or_atm_vol.restype = C.c_double
        L.or_beta_from_atm.argtypes = [C.c_int, _D, _D, _D, _D]
        L.or_atm_seed.argtypes = [C.c_int, C.c_double, C.c_int, C.c_int, _D, _D, C.c_int, _D, _D, _I32, _D, _D,
                                  _D]
        L.or_calibrate.argtypes = [C.POINTER(SAProblem), C.POINTER(SAResult)]
        L.or_calibrate_levels.argtypes = [C.POINTER(SAProblem), C.c_int32, C.c_int32, _D, _D, _D,
                                          _D, _I64, _I64]
        L.or_polish.argtypes = [C.POINTER(SAProblem), _D, _D, _I64]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


# --- random numbers ---------------------------------------------------------
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xffffffff for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xffffffff for v in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def path_normals(seed, scheme, path, step):
    z1, z2 = C.c_double(), C.c_double()
    lib().or_path_normals(seed, scheme, path, step, C.byref(z1), C.byref(z2))
    return z1.value, z2.value


def mc_normals(seed, path, step):
    z1, z2 = C.c_double(), C.c_double()
    lib().or_mc_normals(seed, path, step, C.byref(z1), C.byref(z2))
    return z1.value, z2.value


# --- point formulas ---------------------------------------------------------
def sigma_hagan(K, f, T, alpha, beta, rho, nu):
    return lib().or_sigma_hagan(K, f, T, alpha, beta, rho, nu)


def sigma_obloj(K, f, T, alpha, beta, rho, nu):
    return lib().or_sigma_obloj(K, f, T, alpha, beta, rho, nu)


def sigma_expansion(K, f, T, alpha, beta, rho, nu):
    return lib().or_sigma_expansion(K, f, T, alpha, beta, rho, nu)


def z_over_x(z, rho):
    return lib().or_z_over_x(z, rho)


def case1_integrals(T, nu0, rho0, a, b):
    out = np.zeros(4)
    lib().or_case1_integrals(T, nu0, rho0, a, b, _dp(out))
    return out


def quad_integrals(model, T, rho0, nu0, a, b, drho=0.0, dnu=0.0, qrho=0.0, qnu=0.0):
    p = _f64([rho0, nu0, a, b, drho, dnu, qrho, qnu])
    out = np.zeros(4)
    lib().or_quad_integrals(model, T, _dp(p), _dp(out))
    return out


def sigma_dyn(K, f, T, alpha, beta, ints):
    ints = _f64(ints)
    return lib().or_sigma_dyn(K, f, T, alpha, beta, _dp(ints))


def black_call(F, K, T, sigma, disc=1.0):
    return lib().or_black_call(F, K, T, sigma, disc)


def case2_feasible(x, t_max):
    x = _f64(x)
    return bool(lib().or_case2_feasible(_dp(x), t_max))


# --- grid-level -------------------------------------------------------------
class Market:
    """CSR market grid: maturities T[n], forwards fwd[n], discounts disc[n],
    offsets offs[n+1] and strikes K[offs[n]] with targets target[offs[n]]."""

    def __init__(self, T, fwd, offs, K, target=None, disc=None):
        self.T = _f64(T)
        self.fwd = _f64(fwd)
        self.offs = _i32(offs)
        self.K = _f64(K)
        n = len(self.T)
        self.disc = _f64(disc if disc is not None else np.ones(n))
        self.target = _f64(target if target is not None else np.zeros(len(self.K)))

    @property
    def n_mat(self):
        return len(self.T)

    @property
    def n_obs(self):
        return int(self.offs[-1])


def model_vols(market, model, x, beta, beta_free=False, formula=HAGAN):
    x = _f64(x)
    out = np.zeros(market.n_obs)
    rc = lib().or_model_vols(model, formula, beta, int(beta_free), len(x), _dp(x), market.n_mat,
                             _dp(market.T), _dp(market.fwd), market.offs.ctypes.data_as(_I32),
                             _dp(market.K), _dp(out))
    if rc:
        raise ValueError("or_model_vols failed")
    return out


def objective_formula(market, model, x, beta, beta_free=False, formula=HAGAN, weighting=ABSOLUTE):
    x = _f64(x)
    return lib().or_objective_formula(model, formula, weighting, beta, int(beta_free), len(x), _dp(x),
                                      market.n_mat, _dp(market.T), _dp(market.fwd),
                                      market.offs.ctypes.data_as(_I32), _dp(market.K),
                                      _dp(market.target))


def mc_prices(market, model, x, beta, n_paths, steps_per_year, seed, beta_free=False, scheme=0):
    x = _f64(x)
    price = np.zeros(market.n_obs)
    se = np.zeros(market.n_obs)
    rc = lib().or_mc_prices(model, beta, int(beta_free), len(x), _dp(x), market.n_mat,
                            _dp(market.T), _dp(market.fwd), _dp(market.disc),
                            market.offs.ctypes.data_as(_I32), _dp(market.K), int(n_paths),
                            int(steps_per_year), int(seed), int(scheme), _dp(price), _dp(se))
    if rc:
        raise ValueError("or_mc_prices failed")
    return price, se


def objective_mc(market, model, x, beta, n_paths, steps_per_year, seed, beta_free=False,
                 weighting=RELATIVE, scheme=0):
    x = _f64(x)
    return lib().or_objective_mc(model, weighting, beta, int(beta_free), len(x), _dp(x),
                                 market.n_mat, _dp(market.T), _dp(market.fwd), _dp(market.disc),
                                 market.offs.ctypes.data_as(_I32), _dp(market.K),
                                 _dp(market.target), int(n_paths), int(steps_per_year), int(seed),
                                 int(scheme))


def mc_cliquet(model, x, beta, f0, reset_T, local_floor, local_cap, global_floor, global_cap, n_paths,
               steps_per_year, seed, disc=1.0, beta_free=False, scheme=0):
    """Cliquet price and standard error on the paths of mc_prices."""
    x = _f64(x)
    rt = _f64(reset_T)
    price, se = C.c_double(), C.c_double()
    rc = lib().or_mc_cliquet(model, beta, int(beta_free), len(x), _dp(x), f0, disc, len(rt), _dp(rt),
                             local_floor, local_cap, global_floor, global_cap, int(n_paths), int(steps_per_year),
                             int(seed), int(scheme), C.byref(price), C.byref(se))
    if rc:
        raise ValueError("or_mc_cliquet failed")
    return price.value, se.value


def atm_vol(K, vol, f):
    K, vol = _f64(K), _f64(vol)
    return lib().or_atm_vol(len(K), _dp(K), _dp(vol), f)


def beta_from_atm(fwd, sigma_atm):
    fwd, sa = _f64(fwd), _f64(sigma_atm)
    b, a = C.c_double(), C.c_double()
    if lib().or_beta_from_atm(len(fwd), _dp(fwd), _dp(sa), C.byref(b), C.byref(a)):
        raise ValueError("or_beta_from_atm failed")
    return b.value, a.value


def atm_seed(market, model, lb, ub, beta, beta_free=False):
    """Start point from the at-the-money vols of market.target."""
    lb, ub = _f64(lb), _f64(ub)
    x0 = np.zeros(len(lb))
    rc = lib().or_atm_seed(model, beta, int(beta_free), len(lb), _dp(lb), _dp(ub), market.n_mat, _dp(market.T),
                           _dp(market.fwd), market.offs.ctypes.data_as(_I32), _dp(market.K), _dp(market.target),
                           _dp(x0))
    if rc:
        raise ValueError("or_atm_seed failed")
    return x0


class _Keep:
    pass


def _problem(market, model, lb, ub, beta, n_chains, n_iters, seed, *, beta_free=False,
             formula=HAGAN, weighting=ABSOLUTE, objective=OBJ_FORMULA, chain_len=10, T0=0.0,
             cooling=None, step0=0.1, step_min=1e-4, polish=False, x0=None, mc_paths=0,
             mc_steps_per_year=250, mc_seed=0, mc_scheme=0):
    keep = _Keep()
    keep.lb, keep.ub = _f64(lb), _f64(ub)
    keep.x0 = None if x0 is None else _f64(x0)
    keep.market = market
    if cooling is None:
        cooling = 0.99 ** (1000.0 / n_iters)
    pb = SAProblem(model=model, formula=formula, weighting=weighting, objective=objective,
                   beta=beta, beta_free=int(beta_free), n_par=len(keep.lb), lb=_dp(keep.lb),
                   ub=_dp(keep.ub), x0=(_dp(keep.x0) if keep.x0 is not None else C.cast(None, _D)),
                   n_mat=market.n_mat, T=_dp(market.T), fwd=_dp(market.fwd), disc=_dp(market.disc),
                   offs=market.offs.ctypes.data_as(_I32), K=_dp(market.K),
                   target=_dp(market.target), n_chains=n_chains, n_iters=n_iters,
                   chain_len=chain_len, T0=T0, cooling=cooling, step0=step0, step_min=step_min,
                   seed=seed, polish=int(polish), mc_paths=mc_paths,
                   mc_steps_per_year=mc_steps_per_year, mc_seed=mc_seed, mc_scheme=mc_scheme)
    return pb, keep


def calibrate(market, model, lb, ub, beta, n_chains, n_iters, seed, **kw):
    """Synchronous parallel simulated annealing; returns dict(x, f, ...)."""
    pb, keep = _problem(market, model, lb, ub, beta, n_chains, n_iters, seed, **kw)
    res = SAResult()
    rc = lib().or_calibrate(C.byref(pb), C.byref(res))
    del keep
    if rc:
        raise ValueError("or_calibrate failed: %d" % rc)
    d = pb.n_par
    return dict(x=np.array(res.x[:d]), f=res.f, f_before_polish=res.f_before_polish,
                n_evals=res.n_evals, n_accept=res.n_accept)


def calibrate_levels(market, model, lb, ub, beta, n_chains, n_iters, seed, level_begin, level_end,
                     state, **kw):
    """Run temperature levels [level_begin, level_end) on an explicit chain
    state dict(cx, cf, bx, bf, n_evals, n_accept), updated in place."""
    pb, keep = _problem(market, model, lb, ub, beta, n_chains, n_iters, seed, **kw)
    ne = C.c_int64(state["n_evals"])
    na = C.c_int64(state["n_accept"])
    rc = lib().or_calibrate_levels(C.byref(pb), level_begin, level_end, _dp(state["cx"]),
                                   _dp(state["cf"]), _dp(state["bx"]), _dp(state["bf"]),
                                   C.byref(ne), C.byref(na))
    del keep
    if rc:
        raise ValueError("or_calibrate_levels failed")
    state["n_evals"], state["n_accept"] = ne.value, na.value
    return state
