/*
 * sabr_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, serial, double-precision reference for SABR calibration by
 * synchronous parallel simulated annealing (Fernandez, Ferreiro, Garcia,
 * Leitao, Lopez-Salas, Vazquez: "Static and dynamic SABR stochastic
 * volatility models: calibration and option pricing using GPUs").
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) never links,
 * loads or calls it, and the two share no code.
 *
 * Conventions shared *by specification only* with the GPU library:
 *   parameter vector x = [alpha, rho0, nu0, a, b, d_rho, d_nu, q_rho, q_nu]
 *     static model  : x = [alpha, rho, nu]            (3 entries)
 *     dynamic case I: x = [alpha, rho0, nu0, a, b]      (5 entries)
 *     dynamic case II: all 9 entries
 *     when beta is calibrated it is appended as the last entry.
 *   market grid: CSR by maturity, offs[n_mat+1], strikes K[offs[n_mat]].
 *   random numbers: Philox4x32-10, key = (seed lo, seed hi);
 *     annealing words : counter (chain, iteration, block, 1)
 *     path normals    : counter (path, step/2, 0, 2), words 0,1 for even
 *                       steps and 2,3 for odd steps, u = ((w>>8)+0.5)/2^24,
 *                       Box-Muller (Z1, Z2) = r (cos 2 pi u2, sin 2 pi u2).
 */
#ifndef SABR_ORACLE_H
#define SABR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_STATIC = 0, OR_DYN_I = 1, OR_DYN_II = 2 };
enum { OR_F_HAGAN = 0, OR_F_OBLOJ = 1, OR_F_EXPANSION = 2 };
enum { OR_W_ABSOLUTE = 0, OR_W_RELATIVE = 1 };
enum { OR_OBJ_FORMULA = 0, OR_OBJ_MC = 1 };
enum { OR_MC_PLAIN = 0, OR_MC_ANTITHETIC = 1 };   /* path schemes (antithetic pairs: not in the paper) */

/* random numbers */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_mc_normals(uint64_t seed, int64_t path, int32_t step, double *z1, double *z2);
void or_path_normals(uint64_t seed, int scheme, int64_t path, int32_t step, double *z1, double *z2);

/* implied volatility formulas (one point) */
double or_z_over_x(double z, double rho);
double or_sigma_hagan(double K, double f, double T, double alpha, double beta, double rho, double nu);
double or_sigma_obloj(double K, double f, double T, double alpha, double beta, double rho, double nu);
double or_sigma_expansion(double K, double f, double T, double alpha, double beta, double rho, double nu);
void or_case1_integrals(double T, double nu0, double rho0, double a, double b, double out[4]);
void or_case2_integrals(double T, const double p[8], double out[4]);
void or_quad_integrals(int model, double T, const double p[8], double out[4]);
double or_sigma_dyn(double K, double f, double T, double alpha, double beta, const double ints[4]);
double or_black_call(double F, double K, double T, double sigma, double disc);

/* whole-grid model values: implied vols for the formula objective */
int or_model_vols(int model, int formula, double beta, int beta_free, int n_par, const double *x,
                  int n_mat, const double *T, const double *fwd, const int32_t *offs,
                  const double *K, double *out);

/* objective of the formula technique */
double or_objective_formula(int model, int formula, int weighting, double beta, int beta_free,
                            int n_par, const double *x, int n_mat, const double *T,
                            const double *fwd, const int32_t *offs, const double *K,
                            const double *target);

/* Monte Carlo prices of European calls on one grid (common forward); under */
/* the antithetic scheme n_paths must be even and the standard error comes  */
/* from the pair means */
int or_mc_prices(int model, double beta, int beta_free, int n_par, const double *x,
                 int n_mat, const double *T, const double *fwd, const double *disc,
                 const int32_t *offs, const double *K, int64_t n_paths, int32_t steps_per_year,
                 uint64_t seed, int scheme, double *price, double *std_err);

/* cliquet option with local and global limits (Section 6) on the paths of */
/* or_mc_prices: reset dates reset_T[n_reset] (increasing), returns         */
/* i = 2..n_reset clamped to [local_floor, local_cap], their sum clamped to */
/* [global_floor, global_cap] */
int or_mc_cliquet(int model, double beta, int beta_free, int n_par, const double *x, double f0, double disc,
                  int n_reset, const double *reset_T, double local_floor, double local_cap,
                  double global_floor, double global_cap, int64_t n_paths, int32_t steps_per_year,
                  uint64_t seed, int scheme, double *price, double *std_err);

/* objective of the Monte Carlo technique */
double or_objective_mc(int model, int weighting, double beta, int beta_free, int n_par,
                       const double *x, int n_mat, const double *T, const double *fwd,
                       const double *disc, const int32_t *offs, const double *K,
                       const double *target, int64_t n_paths, int32_t steps_per_year,
                       uint64_t seed, int scheme);

/* at-the-money start point (Section 3): the market vol at K = f of one row, */
/* beta and alpha from a log-log fit of (f, sigma_ATM), the start point x0  */
double or_atm_vol(int m, const double *K, const double *vol, double f);
int or_beta_from_atm(int n, const double *fwd, const double *sigma_atm, double *beta, double *alpha);
int or_atm_seed(int model, double beta, int beta_free, int n_par, const double *lb, const double *ub,
                int n_mat, const double *T, const double *fwd, const int32_t *offs, const double *K,
                const double *target, double *x0);

/* feasibility of case II functional parameters on (0, T_max] */
int or_case2_feasible(const double *x, double t_max);

/* synchronous parallel simulated annealing; returns 0 or a negative code */
typedef struct {
    int32_t model, formula, weighting, objective;
    double beta;
    int32_t beta_free, n_par;
    const double *lb, *ub, *x0;            /* x0 may be NULL: box centre */
    int32_t n_mat;
    const double *T, *fwd, *disc;
    const int32_t *offs;
    const double *K, *target;
    int32_t n_chains, n_iters, chain_len;
    double T0, cooling, step0, step_min;
    uint64_t seed;
    int32_t polish;
    int64_t mc_paths;
    int32_t mc_steps_per_year;
    int32_t mc_scheme;
    uint64_t mc_seed;
} or_sa_problem;

typedef struct {
    double x[10];
    double f;
    double f_before_polish;
    int64_t n_evals;
    int64_t n_accept;
    int32_t status;
} or_sa_result;

int or_calibrate(const or_sa_problem *pb, or_sa_result *res);
/* same, but stops after `n_levels_run` temperature levels and returns the
 * per-chain state, so that a run can be resumed bitwise */
int or_calibrate_levels(const or_sa_problem *pb, int32_t level_begin, int32_t level_end,
                        double *chain_x, double *chain_f, double *best_x, double *best_f,
                        int64_t *n_evals, int64_t *n_accept);
/* Levenberg-Marquardt polish of a formula-objective result */
int or_polish(const or_sa_problem *pb, double *x, double *f, int64_t *n_evals);

#ifdef __cplusplus
}
#endif
#endif
