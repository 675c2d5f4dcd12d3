/*
 * sabr.h -- C ABI of the MI355X SABR calibration library (libsabr_hip.so).
 *
 * What it computes (Fernandez, Ferreiro, Garcia, Leitao, Lopez-Salas,
 * Vazquez, "Static and dynamic SABR stochastic volatility models:
 * calibration and option pricing using GPUs"):
 *   - model implied volatilities of static SABR (Section 2.1: Hagan's
 *     eq. "haganf", Obloj's eq. "sigma-SABR", the expansion eq. "vola_SABR")
 *     and dynamic SABR (Section 2.2: eq. "vola_SABRd" with the functional
 *     parameters of case I, eq. "el_fun_1", or case II, eq. "el_fun_3");
 *   - the market-fit objective of Section 3 (sum of squared absolute or
 *     relative errors, eqs. "error_calibrate_individual_relativo" and
 *     "error_calibrate_relativo");
 *   - European call prices by the log-Euler Monte Carlo scheme of Section 4
 *     (eq. "dis_SABRd", estimator eq. "payoff");
 *   - calibration by synchronous parallel simulated annealing (Section 5,
 *     Techniques I and II).
 *
 * General rules for every entry point
 *   - Plain C99 types only.  Every host array is owned by the caller and is
 *     only read during the call; the library copies what it needs before
 *     returning.  Device memory is owned by the library (or by the caller for
 *     arrays the caller passes as device pointers, see sabr_objective_batch).
 *   - A return value < 0 is an error code (SABR_E_*); a human-readable reason
 *     is kept in the context (sabr_ctx_last_error).  On error no output array
 *     is written except the status fields of results.
 *   - A sabr_ctx is used by one host thread at a time.  All GPU work runs on
 *     the context's stream; blocking calls synchronise that stream before
 *     they return.
 *   - Parameter vector x (doubles):
 *       static         : [alpha, rho, nu]
 *       dynamic case I : [alpha, rho0, nu0, a, b]
 *       dynamic case II: [alpha, rho0, nu0, a, b, d_rho, d_nu, q_rho, q_nu]
 *     with beta appended as a last entry when it is calibrated (beta_free).
 */
#ifndef SABR_H
#define SABR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SABR_OK 0
#define SABR_E_INVAL (-1)      /* an argument is outside its stated domain */
#define SABR_E_NOMEM (-2)      /* host or device allocation failed */
#define SABR_E_BUDGET (-3)     /* the request needs more device memory than the budget */
#define SABR_E_DEVICE (-4)     /* a HIP call failed (message has the HIP error string) */
#define SABR_E_INFEASIBLE (-5) /* case II start point violates rho(t) in [-1,1], nu(t) > 0 */
#define SABR_E_TIMEOUT (-6)    /* a device-side wait exceeded its bound, or poll timed out */
#define SABR_E_CANCELLED (-7)  /* a served request was cancelled */

typedef enum { SABR_STATIC = 0, SABR_DYN_I = 1, SABR_DYN_II = 2 } sabr_model;
typedef enum { SABR_F_HAGAN = 0, SABR_F_OBLOJ = 1, SABR_F_EXPANSION = 2 } sabr_formula;
typedef enum { SABR_OBJ_FORMULA = 0, SABR_OBJ_MC = 1 } sabr_objective;
typedef enum { SABR_W_ABSOLUTE = 0, SABR_W_RELATIVE = 1 } sabr_weighting;
typedef enum { SABR_FP64 = 0, SABR_FP32 = 1 } sabr_precision;

/* Market grid Data_market(K_j, f, T_i), i < n_mat, j < m_i (Section 3),
 * stored by maturity (CSR).  Host arrays.
 *   T[n_mat]      maturities in years, > 0
 *   fwd[n_mat]    forward f_i of maturity i (f = S0 exp((r - y) T)), > 0
 *   disc[n_mat]   discount factor exp(-r T) applied to Monte Carlo prices, > 0
 *                 (may be NULL for formula objectives: 1 is used)
 *   offs[n_mat+1] offs[0] = 0, strictly increasing; row i is offs[i]..offs[i+1]-1
 *   K[n_obs]      strikes (n_obs = offs[n_mat]); > 0 for the formula, >= 0 for MC
 *   target[n_obs] market vols (formula objective) or prices (MC objective);
 *                 finite, and > 0 under relative weighting; may be NULL when
 *                 only model values are wanted. */
typedef struct {
    int32_t n_mat;
    const double *T, *fwd, *disc;
    const int32_t *offs;
    const double *K, *target;
} sabr_market;

/* Model and search box (Sections 2 and 3: beta fixed beforehand or
 * calibrated; Section 5: the annealing starts from a fixed x0).
 *   n_par must equal 3 / 5 / 9 (+1 with beta_free) for the model.
 *   lb[n_par] <= ub[n_par]; rho bounds within [-1, 1]; alpha lb > 0;
 *   beta (fixed) in [0, 1]; x0[n_par] inside the box, or NULL (box centre). */
typedef struct {
    int32_t model;       /* sabr_model */
    double beta;         /* used when beta_free == 0 */
    int32_t beta_free;
    int32_t n_par;
    const double *lb, *ub, *x0;
} sabr_problem;

/* Objective: Technique I (formula; static formulas selectable, dynamic
 * models always use eq. "vola_SABRd") or Technique II (Monte Carlo prices).
 * precision: SABR_FP64 evaluates every formula in double; SABR_FP32 runs
 * the bulk of the formula and path arithmetic in float, with double for the
 * near-the-money z/x(z), the objective sums and the annealing decisions. */
typedef struct {
    int32_t kind;        /* sabr_objective */
    int32_t formula;     /* sabr_formula, static model only */
    int32_t weighting;   /* sabr_weighting */
    int32_t precision;   /* sabr_precision */
} sabr_objspec;

/* Synchronous simulated annealing (Section 5): n_chains Metropolis chains of
 * chain_len iterations per temperature level, then every chain restarts
 * from the best current state.  n_iters iterations per chain in total.
 * T0 <= 0 takes f(x0) (1 if that is not finite and positive).  Level k runs
 * at T0 * c^(k * chain_len) with c = cooling in (0, 1]; proposals move every
 * coordinate by h (2u - 1)(ub - lb), h = max(step0 * sqrt(c^(k chain_len)),
 * step_min), mirrored once at the bound and clamped.  polish != 0 runs a
 * double-precision Levenberg-Marquardt descent from the best state (formula
 * objective only).  Random words: Philox4x32-10 keyed by seed, counter (chain,
 * iteration, block, 1). */
typedef struct {
    int32_t n_chains, n_iters, chain_len;
    double T0, cooling, step0, step_min;
    uint64_t seed;
    int32_t polish;
} sabr_sa;

/* Monte Carlo (Section 4): n_paths paths of the log-Euler scheme with
 * dt = 1/steps_per_year; maturity i is read at step max(1, floor(T_i / dt)).
 * Normals by Box-Muller from Philox4x32-10 keyed by seed, counter
 * (path, step/2, 0, 2).  All maturities of a grid share the paths, so the
 * grid must have a single forward.
 * scheme: SABR_MC_PLAIN, or SABR_MC_ANTITHETIC (variance reduction, not in
 * the paper): paths come in pairs, path 2k drawing counter (k, step/2, 0, 2)
 * and path 2k + 1 the same normals negated; n_paths must be even, prices
 * are the mean over all paths and standard errors come from the n_paths / 2
 * pair means.  Other values are rejected with SABR_E_INVAL; the serving
 * loop takes the plain scheme only. */
enum { SABR_MC_PLAIN = 0, SABR_MC_ANTITHETIC = 1 };
typedef struct {
    int64_t n_paths;
    int32_t steps_per_year;
    uint64_t seed;
    int32_t scheme;      /* last, so that an initialiser of the first three keeps the plain scheme */
} sabr_mc;

typedef struct {
    double x[10];             /* calibrated parameters (n_par used) */
    double f;                 /* objective at x */
    double f_before_polish;   /* best objective found by the annealing */
    int64_t n_evals;          /* objective evaluations (per calibration) */
    int64_t n_accept;         /* accepted Metropolis moves, all chains */
    int32_t status;           /* SABR_OK or an error code */
} sabr_result;

/* One calibration request: its grid, model, objective, annealing schedule
 * and (for the Monte Carlo objective) path settings. */
typedef struct {
    sabr_market market;
    sabr_problem problem;
    sabr_objspec obj;
    sabr_sa sa;
    sabr_mc mc;
} sabr_request;

typedef struct sabr_ctx sabr_ctx;

/* Context on HIP device `device`.  hbm_budget_bytes caps the device memory
 * the library may hold at once (0: no cap).  stream is a hipStream_t (for
 * example PyTorch's current stream) or NULL for a stream of the library's
 * own.  Errors: SABR_E_INVAL (bad device), SABR_E_DEVICE.
 * Environment read here, for tuning and tests: SABR_LANES_PER_CHAIN and
 * SABR_ROW_SPLIT (lane layout of the annealing kernel), SABR_CRN_VARIANT
 * (layout of the Monte Carlo objective kernel), SABR_EXCHANGE_SPINS (polls
 * of a level-end slot before the wait gives up; default 2^22). */
int sabr_ctx_create(int device, size_t hbm_budget_bytes, void *stream, sabr_ctx **out);
void sabr_ctx_destroy(sabr_ctx *ctx);
/* Text of the last error on this context (never NULL; "" when none). */
const char *sabr_ctx_last_error(const sabr_ctx *ctx);
/* Device workspace owned by the caller (for example the memory of a torch
 * tensor on the context's device): while it is set, the context takes every
 * device buffer of sabr_calibrate, sabr_objective_batch and sabr_mc_price
 * from [dev_ptr, dev_ptr + bytes) instead of allocating, starting again at
 * the beginning on each call, and frees the buffers it had allocated.  A call
 * that needs more returns SABR_E_BUDGET.  The caller keeps the memory alive
 * and untouched by other work until the workspace is replaced or the context
 * destroyed.  dev_ptr NULL returns to the library's own allocations.
 * Errors: SABR_E_INVAL (not device memory of the context's device, or fewer
 * than 4096 bytes). */
int sabr_ctx_set_workspace(sabr_ctx *ctx, void *dev_ptr, size_t bytes);
/* Timing of the dominant kernel: with enable != 0 the library brackets each
 * launch of its main kernel (annealing, objective or path kernel) with HIP
 * events on the context's stream; sabr_ctx_timing returns the summed event
 * time and the number of launches since the last reset. */
int sabr_ctx_enable_timing(sabr_ctx *ctx, int enable);
int sabr_ctx_timing(sabr_ctx *ctx, int reset, double *kernel_ms, int64_t *launches,
                    char *kernel_name, size_t name_len);

/* Calibrate one request (Section 5: Technique I with the formula objective,
 * Technique II with Monte Carlo prices): the grid, model and box, objective,
 * annealing schedule and, for the Monte Carlo objective, the path settings
 * (mc may be NULL for the formula objective).  All arguments are host
 * structs read during the call only.  *out receives the calibrated x, f and
 * counters; out->status carries the error code on failure.
 * Errors: SABR_E_INVAL (validation), SABR_E_INFEASIBLE (case II x0 outside
 * the constraints), SABR_E_BUDGET, SABR_E_NOMEM, SABR_E_DEVICE,
 * SABR_E_TIMEOUT (a wait between the workgroups of the request at a level end
 * exceeded its bound; the launch ends early and no result is valid). */
int sabr_calibrate(sabr_ctx *ctx, const sabr_market *market, const sabr_problem *problem, const sabr_objspec *obj,
                   const sabr_sa *sa, const sabr_mc *mc, sabr_result *out);

/* Calibrate n_req independent requests (Section 5, Techniques I and II) in
 * one call: requests with the formula objective run together in one
 * persistent annealing launch per (model, formula, precision) group; Monte
 * Carlo requests run one after the other.  Each result is the one
 * sabr_calibrate gives for the request alone.  out[n_req] receives one
 * result per request (out[r].status < 0 for a request that failed
 * validation; the call then returns SABR_E_INVAL without running anything).
 * Errors as sabr_calibrate. */
int sabr_calibrate_many(sabr_ctx *ctx, int32_t n_req, const sabr_request *reqs, sabr_result *out);

/* Prepared batches (Section 5, Technique I): the same calibration as
 * sabr_calibrate_many for formula-objective requests, split into a setup call
 * that validates the requests, packs their grids, schedules and launch plan
 * and copies them to device memory, and a run call that works only on that
 * device-resident data (grid normalisation, annealing, polish) and copies
 * back the results.  Repeated runs repeat the calibration: a run returns
 * bit for bit what sabr_calibrate_many returns for the same requests.
 *   sabr_batch_prepare: the requests are read during the call only (the
 *     caller may free them on return).  The batch owns its device memory
 *     (not taken from the context's budget or workspace) until
 *     sabr_batch_destroy, and must be destroyed before its context.
 *     Errors: SABR_E_INVAL (a request fails validation, or uses the Monte
 *     Carlo objective), SABR_E_BUDGET, SABR_E_NOMEM, SABR_E_DEVICE.
 *   sabr_batch_run: out[n_req] in request order; runs on the context's
 *     stream and returns when the results are on the host.  Runs of batches
 *     of one context must not overlap (the context is single-threaded).
 *   sabr_batch_destroy: waits for the context's stream and frees the batch
 *     (NULL is ignored). */
typedef struct sabr_batch sabr_batch;
int sabr_batch_prepare(sabr_ctx *ctx, int32_t n_req, const sabr_request *reqs, sabr_batch **out);
int sabr_batch_run(sabr_batch *batch, sabr_result *out);
void sabr_batch_destroy(sabr_batch *batch);

/* Objective at n_x parameter vectors (Section 3 cost functions).
 *   X[n_x * n_par] row-major parameter vectors, f[n_x] objective values,
 *   model[n_x * n_obs] (may be NULL) model vols or prices.
 *   X, f and model may be host or device pointers (each is classified with
 *   hipPointerGetAttributes); device arrays stay where they are.
 *   market.target may be NULL (f is then not written; model must not be NULL).
 *   mc is read only for the Monte Carlo objective.
 * Non-finite or non-positive model vols give f = +inf.  Case II parameter
 * vectors that violate the constraints give f = +inf. */
int sabr_objective_batch(sabr_ctx *ctx, const sabr_market *market, const sabr_problem *problem,
                         const sabr_objspec *obj, const sabr_mc *mc, int64_t n_x,
                         const double *X, double *f, double *model);

/* Monte Carlo prices (Section 4) of the calls on `market` (targets ignored)
 * at the parameters problem->x0 (required), with n_paths paths:
 * price[n_obs] = disc_i * mean(max(F_{M_i} - K, 0)), std_err[n_obs] its
 * standard error (std_err may be NULL).  Host arrays. */
int sabr_mc_price(sabr_ctx *ctx, const sabr_market *market, const sabr_problem *problem,
                  const sabr_mc *mc, int32_t precision, double *price, double *std_err);

/* sabr_mc_price without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, validation and
 * results as sabr_mc_price (bit for bit), but every device buffer of the call
 * (grid, workgroup partial sums, outputs) lives in one static array of 17 MiB
 * that each device holds from the loading of the library until the process
 * ends, and the caller's host arrays are copied to it directly (no pinned
 * staging buffer): the call makes no hipMalloc, hipHostMalloc or hipFree.
 * Limit: the call needs about 32 KiB x n_obs of partial sums (2048
 * workgroups, reached at 2^19 paths) plus 48 bytes per option and maturity,
 * so up to 512 options at any path count (more with fewer paths); larger
 * calls return SABR_E_BUDGET.  Every call on a device shares that device's
 * array: calls that overlap on one device (two host threads, or two contexts
 * on different streams) race and must be serialised by the caller.
 * Errors: as sabr_mc_price, plus SABR_E_BUDGET (too large for the array) and
 * SABR_E_DEVICE (the array's device address could not be obtained). */
int sabr_mc_price_noalloc(sabr_ctx *ctx, const sabr_market *market, const sabr_problem *problem,
                          const sabr_mc *mc, int32_t precision, double *price, double *std_err);

/* At-the-money start point (Section 3, after eq. "sigma-SABR": ln sigma_ATM
 * = ln alpha - (1 - beta) ln f, from the formula at K = f without its
 * T-correction).  market->target holds market vols (> 0; the strikes of each
 * row increasing); x0[n_par] (host) receives: alpha = f_s^(1 - beta)
 * sigma_ATM,s at the shortest maturity s (lowest index on ties), where
 * sigma_ATM of a row is its vol at K = f linear in ln K between the strikes
 * around f (the end strike's vol beyond the row); with beta calibrated and
 * at least two distinct forwards, beta = 1 + the slope of the least-squares
 * line of ln sigma_ATM on ln f over the maturities (otherwise the fixed beta,
 * or the centre of its box); alpha and beta clamped to the box, every other
 * coordinate at the box centre.  problem->x0 is ignored.  The result can be
 * passed back as problem->x0 of a calibration.
 * Errors: SABR_E_INVAL (validation), SABR_E_DEVICE. */
int sabr_atm_seed(sabr_ctx *ctx, const sabr_market *market, const sabr_problem *problem, double *x0);

/* Cliquet price (Section 6, eqs. "eq_cliquet" and "eq:cliquet_global") by
 * the Monte Carlo paths of sabr_mc_price at the parameters problem->x0
 * (required), forward f0 > 0 today, discount factor disc > 0 at expiry.
 * reset_T[n_reset] (years, n_reset >= 2) are the reset dates d_1 < ... < d_D,
 * each read at step max(1, floor(d_i / dt)) of the path grid (the steps must
 * increase).  Payoff per path: the returns R_i = (F(d_i) - F(d_{i-1})) /
 * F(d_{i-1}), i = 2..D, each clamped to [local_floor, local_cap], summed,
 * and the sum clamped to [global_floor, global_cap] (floors <= caps); a
 * return from an absorbed forward is -1.  *price = disc * mean payoff,
 * *std_err its standard error (std_err may be NULL).  Host outputs.
 * Errors: SABR_E_INVAL (validation), SABR_E_DEVICE. */
int sabr_mc_cliquet(sabr_ctx *ctx, const sabr_problem *problem, double f0, double disc, int32_t n_reset,
                    const double *reset_T, double local_floor, double local_cap, double global_floor,
                    double global_cap, const sabr_mc *mc, int32_t precision, double *price, double *std_err);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of calibration requests (Section 5, Techniques
 * I and II, run for many independent requests at once).
 *
 * A worker thread owns a device-resident table of max_slots slots.  A
 * submitted request waits in a queue (first come, first served within each
 * kind) until a slot of its kind is free and its device footprint (grid, schedule, chain state, Monte Carlo
 * partials: 128 KiB per option) fits in the hbm_budget_bytes arena (0: 1 GiB).  Each formula
 * quantum replays a captured HIP graph that normalises new grids, advances
 * every formula slot by up to quantum_levels temperature levels (fewer for
 * slots whose grids make a level costly, so that one large request does not
 * stretch every quantum) and copies the slot states back; beside it, on a second stream, a second captured graph
 * advances every Monte Carlo slot by one iteration and is relaunched at the
 * first quantum boundary after it finishes.  Requests admitted while others run join at the next
 * launch.  Slots 0..max_slots/8-1 take Monte Carlo requests, the others
 * formula requests.
 *
 * Supported requests: FP32 precision, fixed beta, and either the static
 * Hagan formula (<= 256 chains), the dynamic case I formula (<= 512 chains)
 * or the static Monte Carlo objective (<= 64 chains, <= 600 options);
 * grids up to 1024 points and 32 maturities; Monte Carlo requests of at
 * most 131072 paths.  Others: SABR_E_INVAL (use sabr_calibrate).  A
 * request's result depends only on the request (its
 * random words are keyed by its seed and chain ids, its sums run in a fixed
 * order): it is the same alone, in any mix and for any quantum length.
 *
 * Thread safety: submit, poll, cancel and stats may be called from any host
 * thread.  The server uses the context only for its device; it owns its own
 * streams and memory.
 * ------------------------------------------------------------------------- */
typedef struct sabr_server sabr_server;

/* Errors: SABR_E_INVAL (max_slots outside [2, 4096], quantum_levels < 1),
 * SABR_E_NOMEM, SABR_E_DEVICE (graph capture failed). */
int sabr_server_create(sabr_ctx *ctx, int32_t max_slots, size_t hbm_budget_bytes, int32_t quantum_levels,
                       sabr_server **out);
/* Copies the request (the caller may free its arrays on return; mc may be
 * NULL for the formula objective) and queues it; *ticket identifies its
 * result.  Errors: SABR_E_INVAL (invalid or unsupported request, including a
 * Monte Carlo request of more than 131072 paths), SABR_E_BUDGET (larger than
 * the whole budget). */
int sabr_server_submit(sabr_server *srv, const sabr_market *market, const sabr_problem *problem,
                       const sabr_objspec *obj, const sabr_sa *sa, const sabr_mc *mc, uint64_t *ticket);
/* Returns up to max finished requests (tickets[], res[], and, if not NULL,
 * latency_s[] = completion minus submission in seconds), waiting up to
 * timeout_us for the first one.  res[i].status is SABR_OK or
 * SABR_E_CANCELLED.  Returns SABR_E_TIMEOUT if nothing finished in time. */
int sabr_server_poll(sabr_server *srv, int32_t max, int32_t timeout_us, uint64_t *tickets, sabr_result *res,
                     double *latency_s, int32_t *n_done);
/* Cancels a queued or running request (its result comes back cancelled). */
int sabr_server_cancel(sabr_server *srv, uint64_t ticket);
/* Counters since creation (any pointer may be NULL). */
int sabr_server_stats(sabr_server *srv, int64_t *quanta, int64_t *admitted, int64_t *completed, int64_t *queued,
                      int32_t *active, size_t *bytes_in_use, size_t *peak_bytes, int32_t *peak_active);
/* Stops the worker, waits for the current quantum and frees everything;
 * results not yet polled are dropped. */
int sabr_server_destroy(sabr_server *srv);

#ifdef __cplusplus
}
#endif
#endif
