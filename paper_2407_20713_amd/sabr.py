"""Python binding of libsabr_hip.so (include/sabr.h): argument marshalling only.

Every computation runs in the HIP library; if the library is missing this
module raises instead of computing anything itself.  Names follow the C ABI:
sabr_ctx_create, sabr_calibrate, sabr_objective_batch, sabr_mc_price, ...

Host arrays are numpy float64 / int32; device arrays may be passed to
sabr_objective_batch as torch tensors on the GPU (their data pointers go
straight to the library).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsabr_hip.so")

SABR_OK, SABR_E_INVAL, SABR_E_NOMEM, SABR_E_BUDGET = 0, -1, -2, -3
SABR_E_DEVICE, SABR_E_INFEASIBLE, SABR_E_TIMEOUT, SABR_E_CANCELLED = -4, -5, -6, -7
SABR_STATIC, SABR_DYN_I, SABR_DYN_II = 0, 1, 2
SABR_F_HAGAN, SABR_F_OBLOJ, SABR_F_EXPANSION = 0, 1, 2
SABR_OBJ_FORMULA, SABR_OBJ_MC = 0, 1
SABR_MC_PLAIN, SABR_MC_ANTITHETIC = 0, 1
SABR_W_ABSOLUTE, SABR_W_RELATIVE = 0, 1
SABR_FP64, SABR_FP32 = 0, 1

EXPORTED = ["sabr_ctx_create", "sabr_ctx_destroy", "sabr_ctx_last_error", "sabr_ctx_set_workspace",
            "sabr_ctx_enable_timing",
            "sabr_ctx_timing", "sabr_calibrate", "sabr_calibrate_many", "sabr_batch_prepare", "sabr_batch_run",
            "sabr_batch_destroy",
            "sabr_objective_batch", "sabr_mc_price", "sabr_mc_price_noalloc", "sabr_atm_seed", "sabr_mc_cliquet",
            "sabr_server_create", "sabr_server_submit", "sabr_server_poll", "sabr_server_cancel",
            "sabr_server_stats", "sabr_server_destroy"]

_D = C.POINTER(C.c_double)
_I32 = C.POINTER(C.c_int32)


class sabr_market(C.Structure):
    _fields_ = [("n_mat", C.c_int32), ("T", _D), ("fwd", _D), ("disc", _D), ("offs", _I32), ("K", _D),
                ("target", _D)]


class sabr_problem(C.Structure):
    _fields_ = [("model", C.c_int32), ("beta", C.c_double), ("beta_free", C.c_int32), ("n_par", C.c_int32),
                ("lb", _D), ("ub", _D), ("x0", _D)]


class sabr_objspec(C.Structure):
    _fields_ = [("kind", C.c_int32), ("formula", C.c_int32), ("weighting", C.c_int32),
                ("precision", C.c_int32)]


class sabr_sa(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_iters", C.c_int32), ("chain_len", C.c_int32), ("T0", C.c_double),
                ("cooling", C.c_double), ("step0", C.c_double), ("step_min", C.c_double),
                ("seed", C.c_uint64), ("polish", C.c_int32)]


class sabr_mc(C.Structure):
    _fields_ = [("n_paths", C.c_int64), ("steps_per_year", C.c_int32), ("seed", C.c_uint64), ("scheme", C.c_int32)]


class sabr_result(C.Structure):
    _fields_ = [("x", C.c_double * 10), ("f", C.c_double), ("f_before_polish", C.c_double),
                ("n_evals", C.c_int64), ("n_accept", C.c_int64), ("status", C.c_int32)]


class sabr_request(C.Structure):
    _fields_ = [("market", sabr_market), ("problem", sabr_problem), ("obj", sabr_objspec), ("sa", sabr_sa),
                ("mc", sabr_mc)]


class SabrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("sabr error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib(bind_torch_runtime=True):
    """Load libsabr_hip.so; raise if it has not been built.

    PyTorch ships its own HIP runtime under the same soname
    (libamdhip64.so.7).  With bind_torch_runtime (the default) torch is
    imported first, so that this library binds to that runtime and one
    runtime serves torch's memory and streams and this library's kernels
    (the other order leaves torch without a GPU).  Without it the library
    binds to the system runtime, and torch must not be used with the GPU in
    this process."""
    global _lib
    if _lib is None:
        if bind_torch_runtime:
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsabr_hip.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2407_20713_amd.build)")
        L = C.CDLL(LIB_PATH)
        L.sabr_ctx_create.argtypes = [C.c_int, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
        L.sabr_ctx_destroy.argtypes = [C.c_void_p]
        L.sabr_ctx_destroy.restype = None
        L.sabr_ctx_last_error.argtypes = [C.c_void_p]
        L.sabr_ctx_last_error.restype = C.c_char_p
        L.sabr_ctx_set_workspace.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t]
        L.sabr_ctx_enable_timing.argtypes = [C.c_void_p, C.c_int]
        L.sabr_ctx_timing.argtypes = [C.c_void_p, C.c_int, _D, C.POINTER(C.c_int64), C.c_char_p, C.c_size_t]
        L.sabr_calibrate.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem),
                                     C.POINTER(sabr_objspec), C.POINTER(sabr_sa), C.POINTER(sabr_mc),
                                     C.POINTER(sabr_result)]
        L.sabr_calibrate_many.argtypes = [C.c_void_p, C.c_int32, C.POINTER(sabr_request), C.POINTER(sabr_result)]
        L.sabr_batch_prepare.argtypes = [C.c_void_p, C.c_int32, C.POINTER(sabr_request), C.POINTER(C.c_void_p)]
        L.sabr_batch_run.argtypes = [C.c_void_p, C.POINTER(sabr_result)]
        L.sabr_batch_destroy.argtypes = [C.c_void_p]
        L.sabr_batch_destroy.restype = None
        L.sabr_objective_batch.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem),
                                           C.POINTER(sabr_objspec), C.POINTER(sabr_mc), C.c_int64, C.c_void_p,
                                           C.c_void_p, C.c_void_p]
        L.sabr_mc_price.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem),
                                    C.POINTER(sabr_mc), C.c_int32, _D, _D]
        L.sabr_mc_price_noalloc.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem),
                                            C.POINTER(sabr_mc), C.c_int32, _D, _D]
        L.sabr_atm_seed.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem), _D]
        L.sabr_mc_cliquet.argtypes = [C.c_void_p, C.POINTER(sabr_problem), C.c_double, C.c_double, C.c_int32, _D,
                                      C.c_double, C.c_double, C.c_double, C.c_double, C.POINTER(sabr_mc),
                                      C.c_int32, _D, _D]
        L.sabr_server_create.argtypes = [C.c_void_p, C.c_int32, C.c_size_t, C.c_int32, C.POINTER(C.c_void_p)]
        L.sabr_server_submit.argtypes = [C.c_void_p, C.POINTER(sabr_market), C.POINTER(sabr_problem),
                                         C.POINTER(sabr_objspec), C.POINTER(sabr_sa), C.POINTER(sabr_mc),
                                         C.POINTER(C.c_uint64)]
        L.sabr_server_poll.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.POINTER(C.c_uint64),
                                       C.POINTER(sabr_result), _D, C.POINTER(C.c_int32)]
        L.sabr_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
        L.sabr_server_stats.argtypes = [C.c_void_p] + [C.POINTER(C.c_int64)] * 4 + [C.POINTER(C.c_int32)] + \
                                       [C.POINTER(C.c_size_t)] * 2 + [C.POINTER(C.c_int32)]
        L.sabr_server_destroy.argtypes = [C.c_void_p]
        _lib = L
    return _lib


# --- marshalling helpers -------------------------------------------------------
def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _dp(a):
    return a.ctypes.data_as(_D) if a is not None else C.cast(None, _D)


class Market:
    """Host-side grid (keeps the numpy arrays alive while the C struct is used)."""

    def __init__(self, T, fwd, offs, K, target=None, disc=None):
        self.T = _f64(T)
        self.fwd = _f64(fwd)
        self.offs = np.ascontiguousarray(np.asarray(offs, dtype=np.int32))
        self.K = _f64(K)
        self.disc = None if disc is None else _f64(disc)
        self.target = None if target is None else _f64(target)

    @classmethod
    def from_grid(cls, g, target=None):
        return cls(g.T, g.fwd, g.offs, g.K, target=target, disc=g.disc)

    @property
    def n_obs(self):
        return int(self.offs[-1])

    def c(self):
        return sabr_market(len(self.T), _dp(self.T), _dp(self.fwd), _dp(self.disc),
                           self.offs.ctypes.data_as(_I32), _dp(self.K), _dp(self.target))


class Problem:
    def __init__(self, model, beta, lb=None, ub=None, x0=None, beta_free=False, n_par=None):
        self.model, self.beta, self.beta_free = model, float(beta), bool(beta_free)
        self.lb = None if lb is None else _f64(lb)
        self.ub = None if ub is None else _f64(ub)
        self.x0 = None if x0 is None else _f64(x0)
        base = {SABR_STATIC: 3, SABR_DYN_I: 5, SABR_DYN_II: 9}[model]
        self.n_par = n_par if n_par is not None else base + (1 if beta_free else 0)

    def c(self):
        return sabr_problem(self.model, self.beta, int(self.beta_free), self.n_par, _dp(self.lb), _dp(self.ub),
                            _dp(self.x0))


class Ctx:
    """Owning handle of a sabr_ctx."""

    def __init__(self, device=0, hbm_budget_bytes=0, stream=None):
        h = C.c_void_p()
        rc = lib().sabr_ctx_create(device, hbm_budget_bytes, stream, C.byref(h))
        if rc != SABR_OK:
            raise SabrError(rc, "sabr_ctx_create failed")
        self.h = h

    def close(self):
        if self.h:
            for b in list(getattr(self, "batches", ())):
                b.close()
            lib().sabr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc):
        if rc != SABR_OK:
            raise SabrError(rc, lib().sabr_ctx_last_error(self.h).decode())
        return rc


def sabr_ctx_create(device=0, hbm_budget_bytes=0, stream=None):
    return Ctx(device, hbm_budget_bytes, stream)


def sabr_ctx_destroy(ctx):
    ctx.close()


def sabr_ctx_last_error(ctx):
    return lib().sabr_ctx_last_error(ctx.h).decode()


def sabr_ctx_set_workspace(ctx, buf=None, nbytes=None):
    """Let the context take its device buffers from `buf` (a CUDA tensor, kept
    alive by the context handle while set, or a raw device address with
    nbytes); None returns to the library's own allocations."""
    if buf is None:
        ctx.workspace = None
        return ctx.check(lib().sabr_ctx_set_workspace(ctx.h, None, 0))
    if hasattr(buf, "data_ptr"):
        ptr, n = buf.data_ptr(), buf.numel() * buf.element_size()
    else:
        ptr, n = int(buf), int(nbytes)
    rc = ctx.check(lib().sabr_ctx_set_workspace(ctx.h, C.c_void_p(ptr), n if nbytes is None else int(nbytes)))
    ctx.workspace = buf
    return rc


def sabr_ctx_enable_timing(ctx, enable=True):
    ctx.check(lib().sabr_ctx_enable_timing(ctx.h, int(enable)))


def sabr_ctx_timing(ctx, reset=False):
    ms = C.c_double()
    n = C.c_int64()
    name = C.create_string_buffer(64)
    ctx.check(lib().sabr_ctx_timing(ctx.h, int(reset), C.byref(ms), C.byref(n), name, 64))
    return ms.value, n.value, name.value.decode()


class Request:
    """One calibration request (market, problem, objective, annealing, mc)."""

    def __init__(self, market, problem, kind=SABR_OBJ_FORMULA, formula=SABR_F_HAGAN, weighting=SABR_W_ABSOLUTE,
                 precision=SABR_FP64, n_chains=64, n_iters=1000, chain_len=10, T0=0.0, cooling=None, step0=0.1,
                 step_min=1e-4, seed=1, polish=False, n_paths=0, steps_per_year=250, mc_seed=0, mc_scheme=0):
        self.market, self.problem = market, problem
        if cooling is None:
            cooling = 0.99 ** (1000.0 / n_iters)
        self.obj = sabr_objspec(kind, formula, weighting, precision)
        self.sa = sabr_sa(n_chains, n_iters, chain_len, T0, cooling, step0, step_min, seed, int(polish))
        self.mc = sabr_mc(n_paths=n_paths, steps_per_year=steps_per_year, scheme=mc_scheme, seed=mc_seed)

    def c(self):
        return sabr_request(self.market.c(), self.problem.c(), self.obj, self.sa, self.mc)


def sabr_calibrate(ctx, request):
    """Calibrate one Request; returns a dict (x, f, f_before_polish, n_evals, n_accept, status)."""
    m, p = request.market.c(), request.problem.c()
    out = (sabr_result * 1)()
    rc = lib().sabr_calibrate(ctx.h, C.byref(m), C.byref(p), C.byref(request.obj), C.byref(request.sa),
                              C.byref(request.mc), out)
    if rc != SABR_OK:
        raise SabrError(rc, lib().sabr_ctx_last_error(ctx.h).decode())
    return _results([request], out)[0]


def sabr_calibrate_many(ctx, requests):
    """Calibrate a list of Request in one call; returns a list of dicts."""
    n = len(requests)
    arr = (sabr_request * n)(*[r.c() for r in requests])
    out = (sabr_result * n)()
    rc = lib().sabr_calibrate_many(ctx.h, n, arr, out)
    if rc != SABR_OK:
        raise SabrError(rc, lib().sabr_ctx_last_error(ctx.h).decode())
    return _results(requests, out)


def _results(requests, out):
    res = []
    for r, o in zip(requests, out):
        d = r.problem.n_par
        res.append(dict(x=np.array(o.x[:d]), f=o.f, f_before_polish=o.f_before_polish, n_evals=o.n_evals,
                        n_accept=o.n_accept, status=o.status))
    return res


class Batch:
    """Owning handle of a prepared batch (destroyed before its context)."""

    def __init__(self, ctx, requests):
        self.ctx, self.h = ctx, None
        self.requests = list(requests)
        n = len(self.requests)
        arr = (sabr_request * n)(*[r.c() for r in self.requests])
        h = C.c_void_p()
        ctx.check(lib().sabr_batch_prepare(ctx.h, n, arr, C.byref(h)))
        self.h = h
        self.out = (sabr_result * n)()
        if not hasattr(ctx, "batches"):
            import weakref
            ctx.batches = weakref.WeakSet()
        ctx.batches.add(self)

    def close(self):
        if self.h:
            lib().sabr_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sabr_batch_prepare(ctx, requests):
    """Validate and upload a list of formula-objective Request; returns a Batch."""
    return Batch(ctx, requests)


def sabr_batch_run(batch, raw=False):
    """Run a prepared batch; returns a list of dicts like sabr_calibrate (the
    ctypes result array itself with raw=True)."""
    rc = lib().sabr_batch_run(batch.h, batch.out)
    batch.ctx.check(rc)
    return batch.out if raw else _results(batch.requests, batch.out)


def sabr_batch_destroy(batch):
    batch.close()


def _ptr(a):
    """Data pointer of a numpy array or of a torch tensor (host or device)."""
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


def sabr_objective_batch(ctx, market, problem, X, kind=SABR_OBJ_FORMULA, formula=SABR_F_HAGAN,
                         weighting=SABR_W_ABSOLUTE, precision=SABR_FP64, n_paths=0, steps_per_year=250,
                         mc_seed=0, f=None, model=None, want_model=False, mc_scheme=0):
    """Objective at every row of X (numpy or torch, host or device).  Returns (f, model)."""
    is_torch = hasattr(X, "data_ptr")
    if not is_torch:
        X = _f64(X)
    else:
        import torch
        torch.cuda.synchronize()      # tensors filled on torch's stream are complete
    n_x = X.shape[0]
    if f is None and market.target is not None:
        f = np.zeros(n_x) if not is_torch else X.new_zeros(n_x)
    if model is None and want_model:
        model = np.zeros((n_x, market.n_obs)) if not is_torch else X.new_zeros((n_x, market.n_obs))
    m, p = market.c(), problem.c()
    o = sabr_objspec(kind, formula, weighting, precision)
    mc = sabr_mc(n_paths=n_paths, steps_per_year=steps_per_year, scheme=mc_scheme, seed=mc_seed)
    if is_torch:
        torch.cuda.synchronize()      # outputs allocated on torch's stream exist before the library writes
    ctx.check(lib().sabr_objective_batch(ctx.h, C.byref(m), C.byref(p), C.byref(o), C.byref(mc), n_x,
                                         _ptr(X), _ptr(f), _ptr(model)))
    return f, model


def sabr_mc_price(ctx, market, problem, n_paths, steps_per_year=250, seed=0, precision=SABR_FP32, scheme=0):
    """Monte Carlo call prices at problem.x0; returns (price, std_err)."""
    price = np.zeros(market.n_obs)
    se = np.zeros(market.n_obs)
    m, p = market.c(), problem.c()
    mc = sabr_mc(n_paths=n_paths, steps_per_year=steps_per_year, scheme=scheme, seed=seed)
    ctx.check(lib().sabr_mc_price(ctx.h, C.byref(m), C.byref(p), C.byref(mc), precision, _dp(price), _dp(se)))
    return price, se


def sabr_mc_price_noalloc(ctx, market, problem, n_paths, steps_per_year=250, seed=0, precision=SABR_FP32,
                          scheme=0):
    """sabr_mc_price on the library's static device scratch (no device allocation)."""
    price = np.zeros(market.n_obs)
    se = np.zeros(market.n_obs)
    m, p = market.c(), problem.c()
    mc = sabr_mc(n_paths=n_paths, steps_per_year=steps_per_year, scheme=scheme, seed=seed)
    ctx.check(lib().sabr_mc_price_noalloc(ctx.h, C.byref(m), C.byref(p), C.byref(mc), precision, _dp(price),
                                          _dp(se)))
    return price, se


def sabr_atm_seed(ctx, market, problem):
    """At-the-money start point from market.target (market vols); returns x0."""
    x0 = np.zeros(problem.n_par)
    m, p = market.c(), problem.c()
    ctx.check(lib().sabr_atm_seed(ctx.h, C.byref(m), C.byref(p), _dp(x0)))
    return x0


def sabr_mc_cliquet(ctx, problem, f0, reset_T, local_floor, local_cap, global_floor, global_cap, n_paths,
                    steps_per_year=250, seed=0, disc=1.0, precision=SABR_FP32, scheme=0):
    """Cliquet price at problem.x0 on the Monte Carlo paths; returns (price, std_err)."""
    rt = _f64(reset_T)
    price, se = C.c_double(), C.c_double()
    p = problem.c()
    mc = sabr_mc(n_paths=n_paths, steps_per_year=steps_per_year, scheme=scheme, seed=seed)
    ctx.check(lib().sabr_mc_cliquet(ctx.h, C.byref(p), f0, disc, len(rt), _dp(rt), local_floor, local_cap,
                                    global_floor, global_cap, C.byref(mc), precision, C.byref(price),
                                    C.byref(se)))
    return price.value, se.value


# --- serving -------------------------------------------------------------------
class Server:
    """Handle of a sabr_server (continuous batching of calibration requests)."""

    def __init__(self, ctx, max_slots=64, hbm_budget_bytes=0, quantum_levels=10):
        h = C.c_void_p()
        ctx.check(lib().sabr_server_create(ctx.h, max_slots, hbm_budget_bytes, quantum_levels, C.byref(h)))
        self.h, self.ctx = h, ctx

    def submit(self, request):
        t = C.c_uint64()
        m, p = request.market.c(), request.problem.c()
        self.ctx.check(lib().sabr_server_submit(self.h, C.byref(m), C.byref(p), C.byref(request.obj),
                                                C.byref(request.sa), C.byref(request.mc), C.byref(t)))
        return t.value

    def poll(self, max_n=64, timeout_us=0):
        """Finished requests as a list of (ticket, result dict, latency seconds)."""
        tk = (C.c_uint64 * max_n)()
        rs = (sabr_result * max_n)()
        lat = (C.c_double * max_n)()
        n = C.c_int32()
        rc = lib().sabr_server_poll(self.h, max_n, timeout_us, tk, rs, lat, C.byref(n))
        if rc not in (SABR_OK, SABR_E_TIMEOUT):
            raise SabrError(rc, lib().sabr_ctx_last_error(self.ctx.h).decode())
        out = []
        for i in range(n.value):
            o = rs[i]
            out.append((tk[i], dict(x=np.array(o.x[:]), f=o.f, f_before_polish=o.f_before_polish,
                                    n_evals=o.n_evals, n_accept=o.n_accept, status=o.status), lat[i]))
        return out

    def cancel(self, ticket):
        self.ctx.check(lib().sabr_server_cancel(self.h, ticket))

    def stats(self):
        q, a, c, qu = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        act, pa = C.c_int32(), C.c_int32()
        b, pb = C.c_size_t(), C.c_size_t()
        self.ctx.check(lib().sabr_server_stats(self.h, C.byref(q), C.byref(a), C.byref(c), C.byref(qu),
                                               C.byref(act), C.byref(b), C.byref(pb), C.byref(pa)))
        return dict(quanta=q.value, admitted=a.value, completed=c.value, queued=qu.value, active=act.value,
                    bytes_in_use=b.value, peak_bytes=pb.value, peak_active=pa.value)

    def close(self):
        if self.h:
            lib().sabr_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sabr_server_create(ctx, max_slots=64, hbm_budget_bytes=0, quantum_levels=10):
    return Server(ctx, max_slots, hbm_budget_bytes, quantum_levels)


def sabr_server_submit(server, request):
    return server.submit(request)


def sabr_server_poll(server, max_n=64, timeout_us=0):
    return server.poll(max_n, timeout_us)


def sabr_server_cancel(server, ticket):
    server.cancel(ticket)


def sabr_server_stats(server):
    return server.stats()


def sabr_server_destroy(server):
    server.close()
