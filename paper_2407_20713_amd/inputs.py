"""Seeded synthetic inputs: market grids, parameter boxes, parameter draws,
noise and request traces.

This module holds no SABR arithmetic (no implied-vol formula, no path
scheme): it only lays out strikes and maturities and draws random numbers:
the workloads' true parameters and vol noise from Philox4x32-10 streams
(counter (calibration id, redraw, 0, 4) and (point, 0, 0, 3)), the serving
trace from numpy's PCG64.  Model values at the drawn parameters are computed by
whoever uses the grid (the oracle in the tests, the HIP library in the
benchmark), so both sides see the same inputs.

The grids stand in for the paper's market data (EURO STOXX 50 and EUR/USD,
Appendix B: 4 maturities of 19-21 strikes, vols 0.14-0.34); they keep its
shape (a few to 20 maturities, 5-41 strikes, vols 0.1-0.5) and exceed its
sizes.
"""
from dataclasses import dataclass, field

import numpy as np

STATIC, DYN_I, DYN_II = 0, 1, 2
TAG_NOISE, TAG_TRUE = 3, 4


# --- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), for the workloads' draws ---
def philox4x32_10(ctr, key):
    """Philox4x32-10 of counters ctr[..., 4] under key (k0, k1); uint32 words [..., 4]."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4).copy()
    mask = np.uint64(0xFFFFFFFF)
    k0, k1 = np.uint64(key[0]) & mask, np.uint64(key[1]) & mask
    m0, m1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    for _ in range(10):
        p0 = m0 * c[:, 0]
        p1 = m1 * c[:, 2]
        c = np.stack([(p1 >> np.uint64(32)) ^ c[:, 1] ^ k0, p1 & mask,
                      (p0 >> np.uint64(32)) ^ c[:, 3] ^ k1, p0 & mask], axis=1)
        k0 = (k0 + np.uint64(0x9E3779B9)) & mask
        k1 = (k1 + np.uint64(0xBB67AE85)) & mask
    return c.astype(np.uint32).reshape(np.shape(ctr))


def _key(seed):
    return (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF)


class PhiloxStream:
    """Uniforms (w + 1/2) 2^-32 in (0, 1) from Philox4x32-10 under key `seed`:
    the d-th call of random(n) reads the words of counters (stream, d, b, tag),
    b = 0, 1, ... (a redraw takes the next d)."""

    def __init__(self, seed, stream, tag):
        self.key, self.stream, self.tag, self.draw = _key(seed), int(stream), int(tag), 0

    def random(self, n):
        nb = (n + 3) // 4
        ctr = [(self.stream, self.draw, b, self.tag) for b in range(nb)]
        w = philox4x32_10(np.array(ctr, dtype=np.uint64), self.key).ravel()[:n]
        self.draw += 1
        return (w.astype(np.float64) + 0.5) * 2.0 ** -32


@dataclass
class Grid:
    """CSR market grid.  T[n] maturities, fwd[n] forwards, disc[n] discount
    factors, offs[n+1] row offsets, K[offs[n]] strikes."""
    T: np.ndarray
    fwd: np.ndarray
    disc: np.ndarray
    offs: np.ndarray
    K: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_mat(self):
        return len(self.T)

    @property
    def n_obs(self):
        return int(self.offs[-1])


def make_grid(T, strikes_per_maturity, f0=1.0, disc=None):
    """Grid with one forward f0 for every maturity and the given strike rows."""
    T = np.asarray(T, dtype=np.float64)
    rows = [np.asarray(r, dtype=np.float64) for r in strikes_per_maturity]
    offs = np.zeros(len(rows) + 1, dtype=np.int32)
    offs[1:] = np.cumsum([len(r) for r in rows])
    K = np.concatenate(rows) if rows else np.zeros(0)
    fwd = np.full(len(T), float(f0))
    disc = np.ones(len(T)) if disc is None else np.asarray(disc, dtype=np.float64)
    return Grid(T, fwd, disc, offs, K)


# --- parameter boxes ---------------------------------------------------------
def box(model, beta_free=False):
    """Search box: alpha in [0.01, 1], rho in [-0.99, 0.99], nu in [0.01, 2];
    case I adds a, b in [0, 5]; case II adds d_rho, d_nu in [-0.5, 0.5] and
    q_rho, q_nu in [-1, 1]; beta in [0, 1] when calibrated."""
    lb = [0.01, -0.99, 0.01]
    ub = [1.0, 0.99, 2.0]
    if model in (DYN_I, DYN_II):
        lb += [0.0, 0.0]
        ub += [5.0, 5.0]
    if model == DYN_II:
        lb += [-0.5, -0.5, -1.0, -1.0]
        ub += [0.5, 0.5, 1.0, 1.0]
    if beta_free:
        lb += [0.0]
        ub += [1.0]
    return np.array(lb), np.array(ub)


def draw_params(rng, lb, ub):
    """One parameter vector uniform in the box."""
    return lb + (ub - lb) * rng.random(len(lb))


def vol_noise(rng, n, sd=1e-4):
    """Gaussian noise of standard deviation sd (absolute vol).  rng is a
    numpy Generator, or an integer key: then point j takes the first two
    words of Philox4x32-10 at counter (j, 0, 0, 3) as uniforms u1, u2 and
    the Box-Muller normal sqrt(-2 ln u1) cos(2 pi u2)."""
    if isinstance(rng, (int, np.integer)):
        ctr = np.array([(j, 0, 0, TAG_NOISE) for j in range(n)], dtype=np.uint64).reshape(-1, 4)
        w = philox4x32_10(ctr, _key(rng)).astype(np.float64) if n else np.zeros((0, 4))
        u1 = (w[:, 0] + 0.5) * 2.0 ** -32
        u2 = (w[:, 1] + 0.5) * 2.0 ** -32
        return sd * np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return rng.normal(0.0, sd, size=n)


# --- the workloads -----------------------------------------------------------
def single_smile():
    """Static single smile: F0 = 1, T = 1 y, 15 strikes exp(linspace(-0.5, 0.5, 15)),
    beta = 0.7, true (alpha, rho, nu) = (0.2, -0.3, 0.5); 64 chains x 1000
    iterations, cooling 0.99 per iteration."""
    g = make_grid([1.0], [np.exp(np.linspace(-0.5, 0.5, 15))])
    g.meta.update(beta=0.7, x_true=np.array([0.2, -0.3, 0.5]), n_chains=64, n_iters=1000,
                  cooling=0.99, noise_sd=1e-4, noise_seed=0x5AB1, sa_seed=0x5AB10001)
    return g


SURFACE_MATURITIES = np.array([1, 2, 3, 6, 9, 12, 18, 24, 36, 60, 84, 120]) / 12.0


def surface_fits(betas=(0.5, 1.0), n_strikes=25, moneyness=0.6):
    """Static surface: 12 maturities x 25 strikes (log-moneyness +-0.6), each
    maturity fitted on its own, for beta in {0.5, 1.0}: 24 single-maturity
    grids.  4096 chains x 20000 iterations, cooling 0.99^(1000/20000)."""
    fits = []
    strikes = np.exp(np.linspace(-moneyness, moneyness, n_strikes))
    for beta in betas:
        for i, T in enumerate(SURFACE_MATURITIES):
            g = make_grid([T], [strikes])
            g.meta.update(beta=float(beta), fit=len(fits), maturity_index=i)
            fits.append(g)
    return fits


def surface_true_params(n_fits, seed=0x5AB2, model=STATIC):
    """Per-fit stream of true parameters uniform in the box: fit k draws from
    Philox4x32-10 under key `seed` at counter (k, redraw, 0, 4), so a fit whose
    surface is not finite and positive takes the next redraw of its own
    stream."""
    lb, ub = box(model)
    return [PhiloxStream(seed, k, TAG_TRUE) for k in range(n_fits)], lb, ub


def mc_grid(f0=1.0, n_strikes=15, vol_scale=0.2):
    """Monte Carlo objective grid: 8 quarterly maturities 0.25..2 y, strikes
    K_ij = F0 exp(k_j vol_scale sqrt(T_i)), k = linspace(-1.5, 1.5, 15)."""
    T = np.arange(1, 9) * 0.25
    k = np.linspace(-1.5, 1.5, n_strikes)
    rows = [f0 * np.exp(k * vol_scale * np.sqrt(t)) for t in T]
    g = make_grid(T, rows, f0=f0)
    g.meta.update(beta=0.7, x_true=np.array([0.2, -0.3, 0.5]), n_chains=1024, n_iters=500,
                  cooling=0.99 ** 2, paths=65536, steps_per_year=250, target_paths=1 << 22,
                  target_seed=0x5AB37A6E, mc_seed=0x5AB3)
    return g


def dynamic_ladder(n=20):
    """Log-spaced maturities 1 month .. 10 years: T_i = (1/12) 120^(i/(n-1))."""
    return (1.0 / 12.0) * 120.0 ** (np.arange(n) / (n - 1))


def dynamic_surface(n_mat=20, n_strikes=20):
    """Dynamic surface: 20 maturities (1 m - 10 y) x 20 strikes
    exp(linspace(-0.6, 0.6, 20)), joint fit.  Case I true parameters
    (alpha, rho0, nu0, a, b) = (0.2, -0.4, 0.6, 0.3, 0.5), beta = 0.7."""
    strikes = np.exp(np.linspace(-0.6, 0.6, n_strikes))
    g = make_grid(dynamic_ladder(n_mat), [strikes] * n_mat)
    g.meta.update(beta=0.7, x_true=np.array([0.2, -0.4, 0.6, 0.3, 0.5]),
                  x_true_case2=np.array([0.2, -0.4, 0.6, 0.3, 0.5, 0.1, -0.05, 0.2, 0.3]),
                  n_chains=8192, n_iters=50000, cooling=0.99 ** 0.02)
    return g


# --- serving trace -------------------------------------------------------------
@dataclass
class Request:
    arrival_s: float
    kind: str              # "static", "dynamic", "mc"
    grid: Grid
    x_true: np.ndarray
    seed: int
    noise: np.ndarray


def request_trace(n_requests, rate_per_s, seed=0x5AB5, max_mat=20, strike_range=(5, 41),
                  mix=(0.7, 0.2, 0.1), mc_max_T=2.0):
    """Poisson arrivals at rate_per_s; each request draws n_mat ~ U{1..20}
    (the first n_mat maturities of the dynamic ladder, those up to 2 y for
    Monte Carlo requests), n_strike ~ U{5..41} strikes spanning +-0.5
    log-moneyness, a kind by the 70/20/10 mix, true parameters uniform in the
    kind's box, and vol noise of sd 1e-4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    ladder = dynamic_ladder(max_mat)
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        u = rng.random()
        kind = "static" if u < mix[0] else ("dynamic" if u < mix[0] + mix[1] else "mc")
        n_mat = int(rng.integers(1, max_mat + 1))
        T = ladder[:n_mat]
        if kind == "mc":
            T = T[T <= mc_max_T]
            if len(T) == 0:
                T = ladder[:1]
        if kind == "static":
            T = T[-1:]          # one smile per static request
        n_k = int(rng.integers(strike_range[0], strike_range[1] + 1))
        strikes = np.exp(np.linspace(-0.5, 0.5, n_k))
        g = make_grid(T, [strikes] * len(T))
        model = STATIC if kind in ("static", "mc") else DYN_I
        lb, ub = box(model)
        x_true = draw_params(rng, lb, ub)
        noise = vol_noise(rng, g.n_obs)
        out.append(Request(t, kind, g, x_true, int(rng.integers(1, 2 ** 62)), noise))
    return out
