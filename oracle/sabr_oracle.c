/*
 * sabr_oracle.c -- TEST INFRASTRUCTURE ONLY (see sabr_oracle.h).
 *
 * A plain, slow, serial FP64 statement of what the SABR calibration hot path
 * computes, written from the paper's text.  Every function names the passage
 * it follows.  Nothing here is blocked, fused or reordered beyond what the
 * definitions say; quadrature and series are used only where the paper's
 * closed forms cannot be evaluated in floating point (small rate * maturity)
 * or do not exist (case II eta_2^2).
 *
 * Pinned by tests/test_oracle_pins.py against closed forms, limits, printed
 * values and brute force.  The case II integrals are pinned against the
 * closed forms of Appendix A; the paper prints no case II vols to compare
 * end to end.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no -ffast-math),
 * so that the annealing arithmetic is evaluated exactly as written.
 */
#include "sabr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random        */
/* numbers: as easy as 1, 2, 3").  The paper itself draws with XORWOW plus   */
/* Box-Muller (Section 4); a counter-based generator replaces it so that     */
/* every (chain, iteration) and (path, step) owns a fixed set of words.      */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void seed_key(uint64_t seed, uint32_t key[2])
{
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
}

/* Uniform in (0,1) from the top 24 bits: exact in FP32 and FP64. */
static double u24(uint32_t w) { return ((double)(w >> 8) + 0.5) * (1.0 / 16777216.0); }
/* Uniform in (0,1) from a whole word, for the annealing decisions. */
static double u32(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

/* The normals of one step of a path under the path scheme: plain, or       */
/* antithetic pairs, in which paths 2k and 2k + 1 both take the draws of    */
/* counter k and the odd path negates them.                                 */
void or_path_normals(uint64_t seed, int scheme, int64_t path, int32_t step, double *z1, double *z2)
{
    if (scheme == OR_MC_ANTITHETIC) {
        or_mc_normals(seed, path / 2, step, z1, z2);
        if (path % 2 == 1) { *z1 = -*z1; *z2 = -*z2; }
    } else {
        or_mc_normals(seed, path, step, z1, z2);
    }
}

/* Two independent standard normals for one time step of one path, by the   */
/* Box-Muller transform the paper uses (Section 4, GPU process, step 2).    */
void or_mc_normals(uint64_t seed, int64_t path, int32_t step, double *z1, double *z2)
{
    uint32_t key[2], ctr[4], w[4];
    seed_key(seed, key);
    ctr[0] = (uint32_t)path;
    ctr[1] = (uint32_t)(step / 2);
    ctr[2] = 0u;
    ctr[3] = 2u;
    or_philox4x32_10(ctr, key, w);
    double ua = (step % 2 == 0) ? u24(w[0]) : u24(w[2]);
    double ub = (step % 2 == 0) ? u24(w[1]) : u24(w[3]);
    double r = sqrt(-2.0 * log(ua));
    *z1 = r * cos(2.0 * OR_PI * ub);
    *z2 = r * sin(2.0 * OR_PI * ub);
}

/* ------------------------------------------------------------------------ */
/* Static SABR implied volatilities (Section 2.1).                           */
/* ------------------------------------------------------------------------ */

/* z / x(z) with x(z) = ln((sqrt(1 - 2 rho z + z^2) + z - rho) / (1 - rho))  */
/* (eq. "equis").  The argument of the log is 1 + delta with delta formed    */
/* without cancellation: for z - rho < 0 the ratio is rewritten with         */
/* (s + z - rho)(s - z + rho) = 1 - rho^2.  z = 0 gives the limit 1.         */
double or_z_over_x(double z, double rho)
{
    if (z == 0.0) return 1.0;
    double s = sqrt(1.0 - 2.0 * rho * z + z * z);
    double ratio, delta;
    if (z - rho >= 0.0) {
        ratio = (s + z - rho) / (1.0 - rho);
        delta = z * ((z - 2.0 * rho) / (s + 1.0) + 1.0) / (1.0 - rho);
    } else {
        ratio = (1.0 + rho) / (s - z + rho);
        delta = z * ((2.0 * rho - z) / (s + 1.0) + 1.0) / (s - z + rho);
    }
    double x = (fabs(delta) < 0.5) ? log1p(delta) : log(ratio);
    return z / x;
}

/* Hagan's formula, eq. "haganf" with z from eq. "zeta", exactly the printed */
/* terms (the l^4/1920 term included, nothing after the printed dots).      */
double or_sigma_hagan(double K, double f, double T, double alpha, double beta, double rho, double nu)
{
    double omb = 1.0 - beta;
    double l = log(f / K);
    double kf = pow(K * f, omb / 2.0);          /* (K f)^((1-beta)/2) */
    double den = kf * (1.0 + omb * omb / 24.0 * l * l + pow(omb, 4) / 1920.0 * pow(l, 4));
    double z = nu / alpha * kf * l;
    double corr = 1.0 + (omb * omb / 24.0 * alpha * alpha / (kf * kf)
                         + 0.25 * rho * beta * nu * alpha / kf
                         + (2.0 - 3.0 * rho * rho) / 24.0 * nu * nu) * T;
    return alpha / den * or_z_over_x(z, rho) * corr;
}

/* Oblój's correction, eq. "sigma-SABR", as printed: the Hagan denominator    */
/* is kept and the leading factor is nu ln(f/K) / x(z) with                   */
/* z = nu (f^(1-beta) - K^(1-beta)) / (alpha (1-beta)).  The leading factor   */
/* is evaluated as (nu ln(f/K) / z) * (z / x(z)); nu ln(f/K) / z has the      */
/* closed limits alpha (beta = 1) and alpha f^(beta-1) (K = f).               */
double or_sigma_obloj(double K, double f, double T, double alpha, double beta, double rho, double nu)
{
    double omb = 1.0 - beta;
    double l = log(f / K);
    double kf = pow(K * f, omb / 2.0);
    double den = 1.0 + omb * omb / 24.0 * l * l + pow(omb, 4) / 1920.0 * pow(l, 4);
    double z, lead;
    if (fabs(omb) < 1e-8) {
        z = nu / alpha * l;
        lead = alpha;
    } else {
        /* f^(1-beta) - K^(1-beta) = f^(1-beta) * (-expm1((1-beta) ln(K/f))) */
        double diff = pow(f, omb) * (-expm1(omb * log(K / f)));
        z = nu * diff / (alpha * omb);
        lead = (l == 0.0) ? alpha * pow(f, beta - 1.0) : alpha * omb * l / diff;
    }
    double corr = 1.0 + (omb * omb / 24.0 * alpha * alpha / (kf * kf)
                         + 0.25 * rho * beta * nu * alpha / kf
                         + (2.0 - 3.0 * rho * rho) / 24.0 * nu * nu) * T;
    return lead * or_z_over_x(z, rho) / den * corr;
}

/* The second-order expansion, eq. "vola_SABR", with A1, A2, B as printed    */
/* and omega = f^(1-beta) / alpha.                                          */
double or_sigma_expansion(double K, double f, double T, double alpha, double beta, double rho, double nu)
{
    double omb = 1.0 - beta;
    double w = pow(f, omb) / alpha;
    double L = log(K / f);
    double A1 = -0.5 * (omb - rho * nu * w);
    double A2 = (omb * omb + 3.0 * (omb - rho * nu * w) + (2.0 - 3.0 * rho * rho) * nu * nu * w * w) / 12.0;
    double B = omb * omb / 24.0 / (w * w) + beta * rho * nu / 4.0 / w + (2.0 - 3.0 * rho * rho) / 24.0 * nu * nu;
    return (1.0 / w) * (1.0 + A1 * L + A2 * L * L + B * T);
}

/* ------------------------------------------------------------------------ */
/* Dynamic SABR (Section 2.2).                                               */
/* ------------------------------------------------------------------------ */

/* Case I (eq. "el_fun_1"): rho(t) = rho0 e^(-a t), nu(t) = nu0 e^(-b t).     */
/* out = {nu1^2, nu2^2, eta1, eta2^2} of eq. "integrales_SABRd".  The closed  */
/* forms of eq. "exact-integral-expressions" are used when their variable    */
/* (2bT for nu1^2, nu2^2; (a+b)T for eta1, eta2^2) is at least 1; below it    */
/* they cancel, and the Taylor series of the same integrals is summed        */
/* instead (e^(-x u) expanded under the integral sign gives Beta integrals):  */
/*   nu1^2  = nu0^2 sum 6 (-y)^k / (k+3)!                                    */
/*   nu2^2  = nu0^2 sum 6 (k+1) (-y)^k / (k+3)!                              */
/*   eta1   = nu0 rho0 sum 2 (-x)^k / (k+2)!                                 */
/*   eta2^2 = nu0^2 rho0^2 sum 3 (-1)^k (2^(k+4) - 8) x^k / (k+4)!           */
void or_case1_integrals(double T, double nu0, double rho0, double a, double b, double out[4])
{
    double y = 2.0 * b * T;
    double x = (a + b) * T;
    double n1, n2, e1, e2;
    if (fabs(y) >= 1.0) {
        double ey = exp(-y);
        n1 = 6.0 * nu0 * nu0 / (y * y * y) * ((y * y / 2.0 - y + 1.0) - ey);
        n2 = 6.0 * nu0 * nu0 / (y * y * y) * (2.0 * (ey - 1.0) + y * (ey + 1.0));
    } else {
        double s1 = 0.0, s2 = 0.0, fact = 6.0, pw = 1.0; /* fact = (k+3)! */
        for (int k = 0; k < 24; ++k) {
            s1 += 6.0 * pw / fact;
            s2 += 6.0 * (k + 1) * pw / fact;
            pw *= -y;
            fact *= (double)(k + 4);
        }
        n1 = nu0 * nu0 * s1;
        n2 = nu0 * nu0 * s2;
    }
    if (fabs(x) >= 1.0) {
        double ex = exp(-x);
        e1 = 2.0 * nu0 * rho0 / (x * x) * (ex - (1.0 - x));
        e2 = 3.0 * nu0 * nu0 * rho0 * rho0 / (x * x * x * x)
             * (exp(-2.0 * x) - 8.0 * ex + (7.0 + 2.0 * x * (-3.0 + x)));
    } else {
        double s1 = 0.0, s2 = 0.0, f2 = 2.0, f4 = 24.0, pw = 1.0, p2 = 16.0;
        for (int k = 0; k < 24; ++k) {
            s1 += 2.0 * pw / f2;
            s2 += 3.0 * pw * (p2 - 8.0) / f4;
            pw *= -x;
            p2 *= 2.0;
            f2 *= (double)(k + 3);
            f4 *= (double)(k + 5);
        }
        e1 = nu0 * rho0 * s1;
        e2 = nu0 * nu0 * rho0 * rho0 * s2;
    }
    out[0] = n1; out[1] = n2; out[2] = e1; out[3] = e2;
}

/* Functional parameters of eqs. "el_fun_1" and "el_fun_3".                 */
/* p = {rho0, nu0, a, b, d_rho, d_nu, q_rho, q_nu}.                        */
typedef struct { double rho0, nu0, a, b, drho, dnu, qrho, qnu; int model; } fn_params;

static double fn_rho(const fn_params *q, double t)
{
    if (q->model == OR_DYN_I) return q->rho0 * exp(-q->a * t);
    return (q->rho0 + q->qrho * t) * exp(-q->a * t) + q->drho;
}
static double fn_nu(const fn_params *q, double t)
{
    if (q->model == OR_DYN_I) return q->nu0 * exp(-q->b * t);
    return (q->nu0 + q->qnu * t) * exp(-q->b * t) + q->dnu;
}
/* The same sums with every term taken by its magnitude: the size of the     */
/* rounding in fn_rho, fn_nu (eps times this), which where the terms cancel  */
/* is far above eps times the value.                                         */
static double fn_rho_mag(const fn_params *q, double t)
{
    if (q->model == OR_DYN_I) return fabs(q->rho0) * exp(-q->a * t);
    return fabs(q->rho0 + q->qrho * t) * exp(-q->a * t) + fabs(q->drho);
}
static double fn_nu_mag(const fn_params *q, double t)
{
    if (q->model == OR_DYN_I) return fabs(q->nu0) * exp(-q->b * t);
    return fabs(q->nu0 + q->qnu * t) * exp(-q->b * t) + fabs(q->dnu);
}

/* Adaptive Gauss-Legendre quadrature: 10- and 20-point rules on an interval, */
/* bisection until they agree.  Nodes by Newton's method on P_n.             */
static double gl_x10[10], gl_w10[10], gl_x20[20], gl_w20[20];
static int gl_ready = 0;

static void gauss_legendre(int n, double *x, double *w)
{
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            pp = n * (z * p1 - p0) / (z * z - 1.0);
            double z1 = z;
            z = z1 - p1 / pp;
            if (fabs(z - z1) < 1e-16) break;
        }
        x[i] = -z; x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

static void gl_init(void)
{
    if (gl_ready) return;
    gauss_legendre(10, gl_x10, gl_w10);
    gauss_legendre(20, gl_x20, gl_w20);
    gl_ready = 1;
}

typedef double (*integrand_fn)(double t, const void *ctx);

static double gl_rule(integrand_fn g, const void *ctx, double lo, double hi, int n)
{
    const double *xs = n == 10 ? gl_x10 : gl_x20;
    const double *ws = n == 10 ? gl_w10 : gl_w20;
    double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo), s = 0.0;
    for (int i = 0; i < n; ++i) s += ws[i] * g(c + h * xs[i], ctx);
    return s * h;
}

static double integrate(integrand_fn g, const void *ctx, double lo, double hi, double abs_tol, int depth)
{
    double r10 = gl_rule(g, ctx, lo, hi, 10);
    double r20 = gl_rule(g, ctx, lo, hi, 20);
    if (fabs(r20 - r10) <= fmax(1e-14 * fabs(r20), abs_tol) || depth >= 40) return r20;
    double mid = 0.5 * (lo + hi);
    return integrate(g, ctx, lo, mid, 0.5 * abs_tol, depth + 1)
         + integrate(g, ctx, mid, hi, 0.5 * abs_tol, depth + 1);
}

/* Integral of g over [lo, hi] to 1e-14 relative, or, where the integral is */
/* much smaller than its terms (an integrand that changes sign, as nu rho   */
/* does when rho(t) crosses zero), to 1e-14 of the integral of gm, the same */
/* integrand with every term by its magnitude.  The rounding of g is about  */
/* eps gm per value whatever the subinterval, so a purely relative test     */
/* would bisect to the depth limit wherever the terms of g cancel, and      */
/* nested inside eta2^2's outer integral that recursion multiplies out.     */
static double integrate_scaled(integrand_fn g, integrand_fn gm, const void *ctx, double lo, double hi)
{
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    double l1 = 0.0;
    for (int i = 0; i < 20; ++i) l1 += gl_w20[i] * gm(c + h * gl_x20[i], ctx);
    return integrate(g, ctx, lo, hi, 1e-14 * l1 * h + 1e-300, 0);
}

typedef struct { const fn_params *q; double T; } int_ctx;

static double ig_nu1(double t, const void *c)
{ const int_ctx *k = c; double n = fn_nu(k->q, t); return (k->T - t) * (k->T - t) * n * n; }
static double ig_nu1_mag(double t, const void *c)
{ const int_ctx *k = c; double n = fn_nu_mag(k->q, t); return (k->T - t) * (k->T - t) * n * n; }
static double ig_nu2(double t, const void *c)
{ const int_ctx *k = c; double n = fn_nu(k->q, t); return (k->T - t) * t * n * n; }
static double ig_nu2_mag(double t, const void *c)
{ const int_ctx *k = c; double n = fn_nu_mag(k->q, t); return (k->T - t) * t * n * n; }
static double ig_eta1(double t, const void *c)
{ const int_ctx *k = c; return (k->T - t) * fn_nu(k->q, t) * fn_rho(k->q, t); }
static double ig_eta1_mag(double t, const void *c)
{ const int_ctx *k = c; return (k->T - t) * fn_nu_mag(k->q, t) * fn_rho_mag(k->q, t); }
static double ig_nurho(double u, const void *c)
{ const int_ctx *k = c; return fn_nu(k->q, u) * fn_rho(k->q, u); }
static double ig_nurho_mag(double u, const void *c)
{ const int_ctx *k = c; return fn_nu_mag(k->q, u) * fn_rho_mag(k->q, u); }
/* eta2^2's triple integral with the two outer integrals swapped:            */
/* int_0^T int_0^t g(s) ds dt = int_0^T (T - s) g(s) ds, g = I(s)^2 and      */
/* I(s) = int_0^s nu(u) rho(u) du computed by its own quadrature.            */
static double ig_eta2(double s, const void *c)
{
    const int_ctx *k = c;
    double I = (s > 0.0) ? integrate_scaled(ig_nurho, ig_nurho_mag, c, 0.0, s) : 0.0;
    return (k->T - s) * I * I;
}
static double ig_eta2_mag(double s, const void *c)
{
    const int_ctx *k = c;
    double I = (s > 0.0) ? integrate_scaled(ig_nurho_mag, ig_nurho_mag, c, 0.0, s) : 0.0;
    return (k->T - s) * I * I;
}

/* The four integrals of eq. "integrales_SABRd" by quadrature of their       */
/* definitions (case I or case II functional parameters).                    */
void or_quad_integrals(int model, double T, const double p[8], double out[4])
{
    gl_init();
    fn_params q = { p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], model };
    int_ctx c = { &q, T };
    out[0] = 3.0 / (T * T * T) * integrate_scaled(ig_nu1, ig_nu1_mag, &c, 0.0, T);
    out[1] = 6.0 / (T * T * T) * integrate_scaled(ig_nu2, ig_nu2_mag, &c, 0.0, T);
    out[2] = 2.0 / (T * T) * integrate_scaled(ig_eta1, ig_eta1_mag, &c, 0.0, T);
    out[3] = 12.0 / (T * T * T * T) * integrate_scaled(ig_eta2, ig_eta2_mag, &c, 0.0, T);
}

/* Case II: the paper obtains eta2^2 only by quadrature (Section 2.2); the   */
/* other three are computed the same way here.                               */
void or_case2_integrals(double T, const double p[8], double out[4])
{
    or_quad_integrals(OR_DYN_II, T, p, out);
}

/* Osajima's dynamic formula, eq. "vola_SABRd", omega = f^(1-beta) / alpha.   */
double or_sigma_dyn(double K, double f, double T, double alpha, double beta, const double ints[4])
{
    double nu1sq = ints[0], nu2sq = ints[1], eta1 = ints[2], eta2sq = ints[3];
    double omb = 1.0 - beta;
    double w = pow(f, omb) / alpha;
    double L = log(K / f);
    double A1 = (beta - 1.0) / 2.0 + eta1 * w / 2.0;
    double A2 = omb * omb / 12.0 + (1.0 - beta - eta1 * w) / 4.0
              + (4.0 * nu1sq + 3.0 * (eta2sq - 3.0 * eta1 * eta1)) / 24.0 * w * w;
    double B = 1.0 / (w * w) * (omb * omb / 24.0 + w * beta * eta1 / 4.0
                                + (2.0 * nu2sq - 3.0 * eta2sq) / 24.0 * w * w);
    return (1.0 / w) * (1.0 + A1 * L + A2 * L * L + B * T);
}

/* Black's formula for a call on a forward (the pricing the paper applies to */
/* sigma_model when it compares model and market prices, Section 6.2).      */
double or_black_call(double F, double K, double T, double sigma, double disc)
{
    double sd = sigma * sqrt(T);
    if (sd <= 0.0) return disc * fmax(F - K, 0.0);
    double d1 = (log(F / K) + 0.5 * sd * sd) / sd;
    double d2 = d1 - sd;
    double N1 = 0.5 * erfc(-d1 / sqrt(2.0));
    double N2 = 0.5 * erfc(-d2 / sqrt(2.0));
    return disc * (F * N1 - K * N2);
}

/* ------------------------------------------------------------------------ */
/* Parameter vector layout.                                                  */
/* ------------------------------------------------------------------------ */
typedef struct { double alpha, beta, rho0, nu0, a, b, drho, dnu, qrho, qnu; } or_params;

static int expected_npar(int model, int beta_free)
{
    int n = (model == OR_STATIC) ? 3 : (model == OR_DYN_I) ? 5 : (model == OR_DYN_II) ? 9 : -1;
    if (n < 0) return -1;
    return n + (beta_free ? 1 : 0);
}

static int unpack(int model, double beta, int beta_free, int n_par, const double *x, or_params *p)
{
    if (expected_npar(model, beta_free) != n_par) return -1;
    memset(p, 0, sizeof *p);
    p->alpha = x[0]; p->rho0 = x[1]; p->nu0 = x[2];
    if (model != OR_STATIC) { p->a = x[3]; p->b = x[4]; }
    if (model == OR_DYN_II) { p->drho = x[5]; p->dnu = x[6]; p->qrho = x[7]; p->qnu = x[8]; }
    p->beta = beta_free ? x[n_par - 1] : beta;
    return 0;
}

/* Model implied vols over the whole grid (the Data_model of Section 3 with  */
/* Data = implied volatility, Technique I of Section 5).                     */
int or_model_vols(int model, int formula, double beta, int beta_free, int n_par, const double *x,
                  int n_mat, const double *T, const double *fwd, const int32_t *offs,
                  const double *K, double *out)
{
    or_params p;
    if (unpack(model, beta, beta_free, n_par, x, &p)) return -1;
    for (int i = 0; i < n_mat; ++i) {
        double ints[4];
        if (model == OR_DYN_I) or_case1_integrals(T[i], p.nu0, p.rho0, p.a, p.b, ints);
        if (model == OR_DYN_II) {
            double q[8] = { p.rho0, p.nu0, p.a, p.b, p.drho, p.dnu, p.qrho, p.qnu };
            or_case2_integrals(T[i], q, ints);
        }
        for (int j = offs[i]; j < offs[i + 1]; ++j) {
            double s;
            if (model == OR_STATIC) {
                if (formula == OR_F_HAGAN) s = or_sigma_hagan(K[j], fwd[i], T[i], p.alpha, p.beta, p.rho0, p.nu0);
                else if (formula == OR_F_OBLOJ) s = or_sigma_obloj(K[j], fwd[i], T[i], p.alpha, p.beta, p.rho0, p.nu0);
                else s = or_sigma_expansion(K[j], fwd[i], T[i], p.alpha, p.beta, p.rho0, p.nu0);
            } else {
                s = or_sigma_dyn(K[j], fwd[i], T[i], p.alpha, p.beta, ints);
            }
            out[j] = s;
        }
    }
    return 0;
}

/* Squared error of one point: (D_mkt - D_model)^2 (absolute) or            */
/* ((D_mkt - D_model) / D_mkt)^2 as in eqs. "error_calibrate_individual_    */
/* relativo" and "error_calibrate_relativo" (relative).                     */
static double sq_err(int weighting, double target, double model)
{
    double r = target - model;
    if (weighting == OR_W_RELATIVE) { r = r / target; }
    return r * r;
}

/* Objective of Technique I: sum over maturities and strikes of the squared */
/* vol errors.  A model vol that is not finite or not positive makes the    */
/* objective +infinity, so the annealing rejects that point.                */
double or_objective_formula(int model, int formula, int weighting, double beta, int beta_free,
                            int n_par, const double *x, int n_mat, const double *T,
                            const double *fwd, const int32_t *offs, const double *K,
                            const double *target)
{
    int n = offs[n_mat];
    double *m = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!m) return NAN;
    if (or_model_vols(model, formula, beta, beta_free, n_par, x, n_mat, T, fwd, offs, K, m)) {
        free(m);
        return NAN;
    }
    double f = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!isfinite(m[j]) || m[j] <= 0.0) { free(m); return INFINITY; }
        f += sq_err(weighting, target[j], m[j]);
    }
    free(m);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Monte Carlo (Section 4).                                                   */
/* ------------------------------------------------------------------------ */

/* Number of log-Euler steps to maturity T at dt = 1/steps_per_year:        */
/* M = floor(T / dt), at least 1 (the paper's T = 0.495890 gives 123 steps). */
static int32_t n_steps(double T, int32_t spy)
{
    int32_t m = (int32_t)floor(T * (double)spy + 1e-9);
    return m < 1 ? 1 : m;
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } nsum;
static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v)) a->c += (a->s - t) + v;
    else a->c += (v - t) + a->s;
    a->s = t;
}

#define OR_EPS_ABS 1e-30

/* European call prices by the log-Euler scheme of eq. "dis_SABRd", in its   */
/* printed multiplicative form, and the estimator of eq. "payoff".  All     */
/* maturities are read off the same paths at step M_i (common forward).     */
/* A forward that falls below 1e-30 F0 is absorbed at 0.                    */
int or_mc_prices(int model, double beta, int beta_free, int n_par, const double *x,
                 int n_mat, const double *T, const double *fwd, const double *disc,
                 const int32_t *offs, const double *K, int64_t n_paths, int32_t steps_per_year,
                 uint64_t seed, int scheme, double *price, double *std_err)
{
    or_params p;
    if (unpack(model, beta, beta_free, n_par, x, &p)) return -1;
    if (n_paths < 1 || steps_per_year < 1 || n_mat < 1) return -1;
    if (scheme != OR_MC_PLAIN && scheme != OR_MC_ANTITHETIC) return -1;
    if (scheme == OR_MC_ANTITHETIC && n_paths % 2 != 0) return -1;
    for (int i = 1; i < n_mat; ++i) if (fwd[i] != fwd[0]) return -1;
    fn_params q = { p.rho0, p.nu0, p.a, p.b, p.drho, p.dnu, p.qrho, p.qnu, model };
    int n_obs = offs[n_mat];
    int32_t m_max = 0;
    int32_t *mi = malloc(sizeof(int32_t) * (size_t)n_mat);
    nsum *s1 = calloc((size_t)(n_obs > 0 ? n_obs : 1), sizeof(nsum));
    nsum *s2 = calloc((size_t)(n_obs > 0 ? n_obs : 1), sizeof(nsum));
    double *v_even = calloc((size_t)(n_obs > 0 ? n_obs : 1), sizeof(double));   /* first payoff of a pair */
    if (!mi || !s1 || !s2 || !v_even) { free(mi); free(s1); free(s2); free(v_even); return -2; }
    for (int i = 0; i < n_mat; ++i) { mi[i] = n_steps(T[i], steps_per_year); if (mi[i] > m_max) m_max = mi[i]; }
    double dt = 1.0 / (double)steps_per_year;
    double sdt = sqrt(dt);
    double f0 = fwd[0];
    for (int64_t path = 0; path < n_paths; ++path) {
        double al = p.alpha, F = f0;
        int absorbed = 0;
        for (int32_t i = 0; i < m_max; ++i) {
            if (!absorbed) {
                double z1, z2;
                or_path_normals(seed, scheme, path, i, &z1, &z2);
                double t = i * dt;
                double nu = (model == OR_STATIC) ? p.nu0 : fn_nu(&q, t);
                double rho = (model == OR_STATIC) ? p.rho0 : fn_rho(&q, t);
                double nuhat = al * pow(F, p.beta - 1.0);
                double al_next = al * exp(nu * z1 * sdt - nu * nu * dt / 2.0);
                double F_next = F * exp(nuhat * (rho * z1 + z2 * sqrt(1.0 - rho * rho)) * sdt
                                        - nuhat * nuhat * dt / 2.0);
                al = al_next;
                F = F_next;
                if (!(F >= OR_EPS_ABS * f0)) { F = 0.0; absorbed = 1; }
            }
            for (int m = 0; m < n_mat; ++m) {
                if (mi[m] != i + 1) continue;
                for (int j = offs[m]; j < offs[m + 1]; ++j) {
                    double v = fmax(F - K[j], 0.0);
                    if (scheme == OR_MC_ANTITHETIC) {
                        /* one sample per pair: the mean of its two payoffs */
                        if (path % 2 == 0) { v_even[j] = v; continue; }
                        v = 0.5 * (v_even[j] + v);
                    }
                    nsum_add(&s1[j], v);
                    nsum_add(&s2[j], v * v);
                }
            }
        }
    }
    const int64_t n_samp = (scheme == OR_MC_ANTITHETIC) ? n_paths / 2 : n_paths;
    for (int m = 0; m < n_mat; ++m) {
        for (int j = offs[m]; j < offs[m + 1]; ++j) {
            double mean = (s1[j].s + s1[j].c) / (double)n_samp;
            double ex2 = (s2[j].s + s2[j].c) / (double)n_samp;
            double var = (n_samp > 1) ? fmax(ex2 - mean * mean, 0.0) * (double)n_samp / (double)(n_samp - 1) : 0.0;
            price[j] = disc[m] * mean;
            if (std_err) std_err[j] = disc[m] * sqrt(var / (double)n_samp);
        }
    }
    free(mi); free(s1); free(s2); free(v_even);
    return 0;
}

/* Cliquet option (Section 6, pricing with calibrated parameters, eqs.      */
/* "eq_cliquet" and "eq:cliquet_global"): along each path of the scheme of  */
/* eq. "dis_SABRd" (printed multiplicative form, the same normals as        */
/* or_mc_prices) the forward is read at the reset dates d_1 < ... < d_D      */
/* (step max(1, floor(d_i / dt)), as for the European maturities; S_T = F_T, */
/* Section 4), the returns R_i = (F_{d_i} - F_{d_{i-1}}) / F_{d_{i-1}},      */
/* i = 2..D, are clamped to [F_l, C_l] and summed, and the sum is clamped to */
/* [F_g, C_g].  Readings: the printed global payoff max(C_g, min(F_g, .))    */
/* would be the constant C_g whenever F_g < C_g, so the floor and cap are    */
/* read the other way round, max(F_g, min(C_g, .)); a return from an        */
/* absorbed (zero) forward is -1.  price = disc * mean(payoff) (Neumaier     */
/* sums), std_err = disc * sd / sqrt(N).                                    */
int or_mc_cliquet(int model, double beta, int beta_free, int n_par, const double *x, double f0, double disc,
                  int n_reset, const double *reset_T, double local_floor, double local_cap,
                  double global_floor, double global_cap, int64_t n_paths, int32_t steps_per_year,
                  uint64_t seed, int scheme, double *price, double *std_err)
{
    or_params p;
    if (unpack(model, beta, beta_free, n_par, x, &p)) return -1;
    if (n_paths < 1 || steps_per_year < 1 || n_reset < 2 || !(f0 > 0.0)) return -1;
    if (scheme != OR_MC_PLAIN && scheme != OR_MC_ANTITHETIC) return -1;
    if (scheme == OR_MC_ANTITHETIC && n_paths % 2 != 0) return -1;
    fn_params q = { p.rho0, p.nu0, p.a, p.b, p.drho, p.dnu, p.qrho, p.qnu, model };
    int32_t *ms = malloc(sizeof(int32_t) * (size_t)n_reset);
    if (!ms) return -2;
    for (int i = 0; i < n_reset; ++i) {
        ms[i] = n_steps(reset_T[i], steps_per_year);
        if (i > 0 && ms[i] <= ms[i - 1]) { free(ms); return -1; }   /* dates on distinct steps, increasing */
    }
    int32_t m_max = ms[n_reset - 1];
    double dt = 1.0 / (double)steps_per_year;
    double sdt = sqrt(dt);
    nsum s1 = { 0.0, 0.0 }, s2 = { 0.0, 0.0 };
    double v_even = 0.0;   /* first payoff of an antithetic pair */
    for (int64_t path = 0; path < n_paths; ++path) {
        double al = p.alpha, F = f0;
        int absorbed = 0, next = 0;
        double F_prev = 0.0, sum = 0.0;
        for (int32_t i = 0; i < m_max; ++i) {
            if (!absorbed) {
                double z1, z2;
                or_path_normals(seed, scheme, path, i, &z1, &z2);
                double t = i * dt;
                double nu = (model == OR_STATIC) ? p.nu0 : fn_nu(&q, t);
                double rho = (model == OR_STATIC) ? p.rho0 : fn_rho(&q, t);
                double nuhat = al * pow(F, p.beta - 1.0);
                double al_next = al * exp(nu * z1 * sdt - nu * nu * dt / 2.0);
                double F_next = F * exp(nuhat * (rho * z1 + z2 * sqrt(1.0 - rho * rho)) * sdt
                                        - nuhat * nuhat * dt / 2.0);
                al = al_next;
                F = F_next;
                if (!(F >= OR_EPS_ABS * f0)) { F = 0.0; absorbed = 1; }
            }
            if (next < n_reset && ms[next] == i + 1) {
                if (next > 0) {
                    double R = (F_prev > 0.0) ? (F - F_prev) / F_prev : -1.0;
                    sum += fmax(fmin(R, local_cap), local_floor);
                }
                F_prev = F;
                ++next;
            }
        }
        double v = fmax(global_floor, fmin(global_cap, sum));
        if (scheme == OR_MC_ANTITHETIC) {
            if (path % 2 == 0) { v_even = v; continue; }
            v = 0.5 * (v_even + v);
        }
        nsum_add(&s1, v);
        nsum_add(&s2, v * v);
    }
    const int64_t n_samp = (scheme == OR_MC_ANTITHETIC) ? n_paths / 2 : n_paths;
    double mean = (s1.s + s1.c) / (double)n_samp;
    double ex2 = (s2.s + s2.c) / (double)n_samp;
    double var = (n_samp > 1) ? fmax(ex2 - mean * mean, 0.0) * (double)n_samp / (double)(n_samp - 1) : 0.0;
    *price = disc * mean;
    if (std_err) *std_err = disc * sqrt(var / (double)n_samp);
    free(ms);
    return 0;
}

/* Objective of Technique II: relative (or absolute) squared price errors   */
/* with Monte Carlo model prices on fixed paths (common random numbers).    */
double or_objective_mc(int model, int weighting, double beta, int beta_free, int n_par,
                       const double *x, int n_mat, const double *T, const double *fwd,
                       const double *disc, const int32_t *offs, const double *K,
                       const double *target, int64_t n_paths, int32_t steps_per_year,
                       uint64_t seed, int scheme)
{
    int n = offs[n_mat];
    double *m = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!m) return NAN;
    if (or_mc_prices(model, beta, beta_free, n_par, x, n_mat, T, fwd, disc, offs, K, n_paths,
                     steps_per_year, seed, scheme, m, NULL)) { free(m); return NAN; }
    double f = 0.0;
    for (int j = 0; j < n; ++j) {
        if (!isfinite(m[j])) { free(m); return INFINITY; }
        f += sq_err(weighting, target[j], m[j]);
    }
    free(m);
    return f;
}

/* ------------------------------------------------------------------------ */
/* Start point from the at-the-money vols (Section 3, after eq. "sigma-SABR"):*/
/* sigma_ATM = sigma_model(f, f, T) gives ln sigma_ATM = ln alpha            */
/* - (1 - beta) ln f, so beta is the slope + 1 of a log-log least-squares    */
/* fit of sigma_ATM against f, and, with B T neglected,                      */
/* alpha = f^(1 - beta) sigma_ATM.                                           */
/* Readings: sigma_ATM of maturity i is the market vol at K = f_i, linear in */
/* ln K between the two strikes around f_i (the nearest strike's vol beyond  */
/* the row's ends); beta is estimated only when it is calibrated and the     */
/* grid has at least two distinct forwards (otherwise the fixed beta, or the */
/* centre of its box); alpha comes from the shortest maturity, where the     */
/* neglected B T is smallest; alpha and beta are clamped to their box; every */
/* other coordinate is the box centre.                                       */
/* ------------------------------------------------------------------------ */
double or_atm_vol(int m, const double *K, const double *vol, double f)
{
    /* strikes of a row are increasing */
    if (f <= K[0]) return vol[0];
    if (f >= K[m - 1]) return vol[m - 1];
    int j = 0;
    while (K[j + 1] < f) ++j;
    double u = (log(f) - log(K[j])) / (log(K[j + 1]) - log(K[j]));
    return vol[j] + u * (vol[j + 1] - vol[j]);
}

int or_beta_from_atm(int n, const double *fwd, const double *sigma_atm, double *beta, double *alpha)
{
    /* least squares of ln sigma = c0 + c1 ln f: beta = 1 + c1, alpha = e^c0 */
    if (n < 2) return -1;
    double mx = 0.0, my = 0.0;
    for (int i = 0; i < n; ++i) { mx += log(fwd[i]); my += log(sigma_atm[i]); }
    mx /= n; my /= n;
    double sxx = 0.0, sxy = 0.0;
    for (int i = 0; i < n; ++i) {
        double dx = log(fwd[i]) - mx;
        sxx += dx * dx;
        sxy += dx * (log(sigma_atm[i]) - my);
    }
    if (!(sxx > 0.0)) return -1;
    double c1 = sxy / sxx;
    *beta = 1.0 + c1;
    *alpha = exp(my - c1 * mx);
    return 0;
}

int or_atm_seed(int model, double beta, int beta_free, int n_par, const double *lb, const double *ub,
                int n_mat, const double *T, const double *fwd, const int32_t *offs, const double *K,
                const double *target, double *x0)
{
    if (expected_npar(model, beta_free) != n_par || n_mat < 1) return -1;
    for (int k = 0; k < n_par; ++k) x0[k] = 0.5 * (lb[k] + ub[k]);
    double *sa = malloc(sizeof(double) * (size_t)n_mat);
    if (!sa) return -2;
    int shortest = 0, distinct = 0;
    for (int i = 0; i < n_mat; ++i) {
        sa[i] = or_atm_vol(offs[i + 1] - offs[i], K + offs[i], target + offs[i], fwd[i]);
        if (T[i] < T[shortest]) shortest = i;
        if (fwd[i] != fwd[0]) distinct = 1;
    }
    double b = beta;
    if (beta_free) {
        double bb, aa;
        b = x0[n_par - 1];
        if (distinct && or_beta_from_atm(n_mat, fwd, sa, &bb, &aa) == 0)
            b = fmin(fmax(bb, lb[n_par - 1]), ub[n_par - 1]);
        x0[n_par - 1] = b;
    }
    double a = pow(fwd[shortest], 1.0 - b) * sa[shortest];
    x0[0] = fmin(fmax(a, lb[0]), ub[0]);
    free(sa);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Case II constraints (Section 5, Technique II): rho(t) in [-1, 1] and      */
/* nu(t) > 0 for every 0 < t <= T_max.  Each function is (c0 + c1 t) e^(-k t) */
/* + d; its extrema on [0, T_max] lie at the ends or at the one stationary   */
/* point t* = 1/k - c0/c1 (k != 0, c1 != 0; the derivative e^(-k t) (c1 -     */
/* k (c0 + c1 t)) vanishes there whatever the sign of k, so growing as well  */
/* as decaying exponentials are covered).  The value at t = 0 stands for     */
/* the limit t -> 0+.                                                         */
/* ------------------------------------------------------------------------ */
static void fn_extrema(double c0, double c1, double k, double d, double tmax, double *lo, double *hi)
{
    double v0 = c0 + d, v1 = (c0 + c1 * tmax) * exp(-k * tmax) + d;
    *lo = fmin(v0, v1); *hi = fmax(v0, v1);
    if (k != 0.0 && c1 != 0.0) {
        double ts = 1.0 / k - c0 / c1;
        if (ts > 0.0 && ts < tmax) {
            double v = (c0 + c1 * ts) * exp(-k * ts) + d;
            *lo = fmin(*lo, v); *hi = fmax(*hi, v);
        }
    }
}

int or_case2_feasible(const double *x, double t_max)
{
    /* x = [alpha, rho0, nu0, a, b, d_rho, d_nu, q_rho, q_nu] */
    double rlo, rhi, nlo, nhi;
    fn_extrema(x[1], x[7], x[3], x[5], t_max, &rlo, &rhi);
    fn_extrema(x[2], x[8], x[4], x[6], t_max, &nlo, &nhi);
    return (rlo >= -1.0 && rhi <= 1.0 && nlo > 0.0) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Synchronous parallel simulated annealing (Section 5, Technique I).        */
/*                                                                          */
/* Reading of the unstated details (the paper gives only: fixed start x0,   */
/* chains of constant length L at a fixed temperature, then the argmin      */
/* over the chains' final states restarts every chain):                     */
/*   x0 = box centre unless given; T0 = f(x0) unless given (1 if f(x0) is   */
/*   not finite and positive); level k runs iterations kL .. kL+L-1 at      */
/*   T_k = T0 g_k with g_0 = 1, g_(k+1) = g_k * c^L (c the per-iteration    */
/*   cooling factor); step h_k = max(step0 sqrt(g_k), step_min);             */
/*   proposal y = x + h (2u - 1)(ub - lb) on every coordinate, mirrored once */
/*   at the bound it crosses and then clamped; accept if f(y) <= f(x) or    */
/*   u < exp(-(f(y) - f(x)) / T_k); best-so-far over every accepted state;  */
/*   level-end argmin over current states, ties to the lowest chain index.  */
/* ------------------------------------------------------------------------ */
static double eval_objective(const or_sa_problem *pb, const double *x)
{
    double f;
    if (pb->model == OR_DYN_II) {
        double tmax = 0.0;
        for (int i = 0; i < pb->n_mat; ++i) tmax = fmax(tmax, pb->T[i]);
        if (!or_case2_feasible(x, tmax)) return INFINITY;
    }
    if (pb->objective == OR_OBJ_FORMULA)
        f = or_objective_formula(pb->model, pb->formula, pb->weighting, pb->beta, pb->beta_free,
                                 pb->n_par, x, pb->n_mat, pb->T, pb->fwd, pb->offs, pb->K, pb->target);
    else
        f = or_objective_mc(pb->model, pb->weighting, pb->beta, pb->beta_free, pb->n_par, x,
                            pb->n_mat, pb->T, pb->fwd, pb->disc, pb->offs, pb->K, pb->target,
                            pb->mc_paths, pb->mc_steps_per_year, pb->mc_seed, pb->mc_scheme);
    if (!(f == f)) f = INFINITY;  /* NaN ranks last */
    return f;
}

static double propose(double x, double u, double h, double lb, double ub)
{
    double y = x + (h * (2.0 * u - 1.0)) * (ub - lb);
    if (y > ub) y = ub - (y - ub);
    if (y < lb) y = lb + (lb - y);
    if (y > ub) y = ub;
    if (y < lb) y = lb;
    return y;
}

static void start_point(const or_sa_problem *pb, double *x0)
{
    for (int j = 0; j < pb->n_par; ++j)
        x0[j] = pb->x0 ? pb->x0[j] : 0.5 * (pb->lb[j] + pb->ub[j]);
}

static double start_temperature(const or_sa_problem *pb, const double *x0)
{
    if (pb->T0 > 0.0) return pb->T0;
    double f0 = eval_objective(pb, x0);
    return (isfinite(f0) && f0 > 0.0) ? f0 : 1.0;
}

int or_calibrate_levels(const or_sa_problem *pb, int32_t level_begin, int32_t level_end,
                        double *cx, double *cf, double *bx, double *bf,
                        int64_t *n_evals, int64_t *n_accept)
{
    int d = pb->n_par, P = pb->n_chains, L = pb->chain_len;
    if (d < 1 || d > 10 || P < 1 || L < 1 || pb->n_iters < 1) return -1;
    double x0[10];
    start_point(pb, x0);
    double T0 = start_temperature(pb, x0);
    double cL = pow(pb->cooling, (double)L);
    double g = 1.0;
    for (int32_t k = 0; k < level_begin; ++k) g = g * cL;
    int32_t n_levels = (pb->n_iters + L - 1) / L;
    uint32_t key[2];
    seed_key(pb->seed, key);
    double y[10];
    for (int32_t k = level_begin; k < level_end && k < n_levels; ++k) {
        double Tk = T0 * g;
        double h = fmax(pb->step0 * sqrt(g), pb->step_min);
        for (int p = 0; p < P; ++p) {
            double *x = cx + (size_t)p * d;
            for (int32_t t = k * L; t < (k + 1) * L && t < pb->n_iters; ++t) {
                double u[12];
                for (int blk = 0; blk * 4 < d + 1; ++blk) {
                    uint32_t ctr[4] = { (uint32_t)p, (uint32_t)t, (uint32_t)blk, 1u }, w[4];
                    or_philox4x32_10(ctr, key, w);
                    for (int q = 0; q < 4; ++q) u[blk * 4 + q] = u32(w[q]);
                }
                for (int j = 0; j < d; ++j) y[j] = propose(x[j], u[j], h, pb->lb[j], pb->ub[j]);
                double fy = eval_objective(pb, y);
                ++*n_evals;
                double delta = fy - cf[p];
                if (delta <= 0.0 || u[d] < exp(-delta / Tk)) {
                    memcpy(x, y, sizeof(double) * (size_t)d);
                    cf[p] = fy;
                    ++*n_accept;
                    if (fy < bf[p]) { memcpy(bx + (size_t)p * d, y, sizeof(double) * (size_t)d); bf[p] = fy; }
                }
            }
        }
        /* level end: every chain restarts from the best current state */
        int best = 0;
        for (int p = 1; p < P; ++p) if (cf[p] < cf[best]) best = p;
        for (int p = 0; p < P; ++p) {
            if (p == best) continue;
            memcpy(cx + (size_t)p * d, cx + (size_t)best * d, sizeof(double) * (size_t)d);
            cf[p] = cf[best];
        }
        g = g * cL;
    }
    return 0;
}

/* Residual vector of the formula objective: r_j = (D_mkt - D_model) * s_j  */
/* with s_j = 1 (absolute) or 1/D_mkt (relative), so that f = sum r_j^2.     */
/* Returns 0 if every model value is finite and positive.                    */
static int residuals(const or_sa_problem *pb, const double *x, double *r)
{
    int n = pb->offs[pb->n_mat];
    if (pb->model == OR_DYN_II) {
        double tmax = 0.0;
        for (int i = 0; i < pb->n_mat; ++i) tmax = fmax(tmax, pb->T[i]);
        if (!or_case2_feasible(x, tmax)) return -1;
    }
    if (or_model_vols(pb->model, pb->formula, pb->beta, pb->beta_free, pb->n_par, x, pb->n_mat, pb->T,
                      pb->fwd, pb->offs, pb->K, r)) return -1;
    for (int j = 0; j < n; ++j) {
        if (!isfinite(r[j]) || r[j] <= 0.0) return -1;
        double e = pb->target[j] - r[j];
        r[j] = (pb->weighting == OR_W_RELATIVE) ? e / pb->target[j] : e;
    }
    return 0;
}

static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Solve (A + lambda D) d = -g by Cholesky, A symmetric d x d (row-major),   */
/* D = diag(A) floored at 1e-12 of its mean.  Returns 0 on success.          */
static int damped_solve(int d, const double *A, const double *g, double lambda, double *delta)
{
    double M[100], L[100], y[10], tr = 0.0;
    for (int k = 0; k < d; ++k) tr += A[k * d + k];
    double floor_ = 1e-12 * tr / d + 1e-300;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) M[a * d + b] = A[a * d + b];
    for (int k = 0; k < d; ++k) M[k * d + k] += lambda * fmax(A[k * d + k], floor_);
    for (int a = 0; a < d; ++a) {
        for (int b = 0; b <= a; ++b) {
            double s = M[a * d + b];
            for (int k = 0; k < b; ++k) s -= L[a * d + k] * L[b * d + k];
            if (a == b) {
                if (!(s > 0.0)) return -1;
                L[a * d + a] = sqrt(s);
            } else {
                L[a * d + b] = s / L[b * d + b];
            }
        }
    }
    for (int a = 0; a < d; ++a) {          /* L y = -g */
        double s = -g[a];
        for (int k = 0; k < a; ++k) s -= L[a * d + k] * y[k];
        y[a] = s / L[a * d + a];
    }
    for (int a = d - 1; a >= 0; --a) {     /* L^T delta = y */
        double s = y[a];
        for (int k = a + 1; k < d; ++k) s -= L[k * d + a] * delta[k];
        delta[a] = s / L[a * d + a];
    }
    return 0;
}

/* Levenberg-Marquardt polish of the annealing result (reading of the      */
/* "best-so-far polish"), double precision, formula objective:             */
/*   Jacobian of the residuals by central differences with steps            */
/*   h_k = 6e-6 (ub_k - lb_k), clamped to the box;                           */
/*   step: (J^T J + lambda diag(J^T J)) delta = -J^T r, y = clamp(x + delta);*/
/*   accept if f(y) < f(x) (lambda /= 10, at least 1e-15), else lambda *= 10 */
/*   and retry up to 12 times; lambda starts at 1e-3;                        */
/*   at most 60 iterations; stops when f = 0, when no damping improves f,    */
/*   or when an accepted step lowers f by less than 1e-15 f.                 */
int or_polish(const or_sa_problem *pb, double *x, double *f, int64_t *n_evals)
{
    int d = pb->n_par, n = pb->offs[pb->n_mat];
    double *r = malloc(sizeof(double) * (size_t)n), *rp = malloc(sizeof(double) * (size_t)n);
    double *rm = malloc(sizeof(double) * (size_t)n), *J = malloc(sizeof(double) * (size_t)n * d);
    if (!r || !rp || !rm || !J) { free(r); free(rp); free(rm); free(J); return -2; }
    double lambda = 1e-3;
    if (residuals(pb, x, r)) { free(r); free(rp); free(rm); free(J); return 0; }
    double fx = 0.0;
    for (int j = 0; j < n; ++j) fx += r[j] * r[j];
    ++*n_evals;
    for (int it = 0; it < 60 && fx > 0.0; ++it) {
        for (int k = 0; k < d; ++k) {
            double h = 6e-6 * (pb->ub[k] - pb->lb[k]);
            double xp[10], xm[10];
            memcpy(xp, x, sizeof(double) * (size_t)d);
            memcpy(xm, x, sizeof(double) * (size_t)d);
            xp[k] = clampd(x[k] + h, pb->lb[k], pb->ub[k]);
            xm[k] = clampd(x[k] - h, pb->lb[k], pb->ub[k]);
            double den = xp[k] - xm[k];
            int bad = residuals(pb, xp, rp) | residuals(pb, xm, rm);
            *n_evals += 2;
            for (int j = 0; j < n; ++j) J[(size_t)j * d + k] = (den > 0.0 && !bad) ? (rp[j] - rm[j]) / den : 0.0;
        }
        double A[100], g[10];
        for (int a = 0; a < d; ++a) {
            g[a] = 0.0;
            for (int j = 0; j < n; ++j) g[a] += J[(size_t)j * d + a] * r[j];
            for (int b = 0; b < d; ++b) {
                double s = 0.0;
                for (int j = 0; j < n; ++j) s += J[(size_t)j * d + a] * J[(size_t)j * d + b];
                A[a * d + b] = s;
            }
        }
        int moved = 0;
        double fnew = fx;
        for (int tries = 0; tries < 12; ++tries) {
            double delta[10], y[10];
            if (damped_solve(d, A, g, lambda, delta) == 0) {
                for (int k = 0; k < d; ++k) y[k] = clampd(x[k] + delta[k], pb->lb[k], pb->ub[k]);
                ++*n_evals;
                if (residuals(pb, y, rp) == 0) {
                    double fy = 0.0;
                    for (int j = 0; j < n; ++j) fy += rp[j] * rp[j];
                    if (fy < fx) {
                        memcpy(x, y, sizeof(double) * (size_t)d);
                        memcpy(r, rp, sizeof(double) * (size_t)n);
                        fnew = fy;
                        lambda = fmax(lambda / 10.0, 1e-15);
                        moved = 1;
                        break;
                    }
                }
            }
            lambda *= 10.0;
        }
        if (!moved) break;
        double gain = fx - fnew;
        fx = fnew;
        if (gain <= 1e-15 * fx) break;
    }
    *f = fx;
    free(r); free(rp); free(rm); free(J);
    return 0;
}

int or_calibrate(const or_sa_problem *pb, or_sa_result *res)
{
    int d = pb->n_par, P = pb->n_chains;
    memset(res, 0, sizeof *res);
    if (expected_npar(pb->model, pb->beta_free) != d || P < 1 || pb->chain_len < 1 || pb->n_iters < 1) {
        res->status = -1;
        return -1;
    }
    double x0[10];
    start_point(pb, x0);
    double f0 = eval_objective(pb, x0);
    double *cx = malloc(sizeof(double) * (size_t)P * d), *bx = malloc(sizeof(double) * (size_t)P * d);
    double *cf = malloc(sizeof(double) * (size_t)P), *bf = malloc(sizeof(double) * (size_t)P);
    if (!cx || !bx || !cf || !bf) { free(cx); free(bx); free(cf); free(bf); res->status = -2; return -2; }
    for (int p = 0; p < P; ++p) {
        memcpy(cx + (size_t)p * d, x0, sizeof(double) * (size_t)d);
        memcpy(bx + (size_t)p * d, x0, sizeof(double) * (size_t)d);
        cf[p] = f0; bf[p] = f0;
    }
    int64_t ne = 1, na = 0;
    int32_t n_levels = (pb->n_iters + pb->chain_len - 1) / pb->chain_len;
    int rc = or_calibrate_levels(pb, 0, n_levels, cx, cf, bx, bf, &ne, &na);
    if (rc) { free(cx); free(bx); free(cf); free(bf); res->status = rc; return rc; }
    int best = 0;
    for (int p = 1; p < P; ++p) if (bf[p] < bf[best]) best = p;
    memcpy(res->x, bx + (size_t)best * d, sizeof(double) * (size_t)d);
    res->f = bf[best];
    res->f_before_polish = bf[best];
    if (pb->polish && pb->objective == OR_OBJ_FORMULA) or_polish(pb, res->x, &res->f, &ne);
    res->n_evals = ne;
    res->n_accept = na;
    res->status = 0;
    free(cx); free(bx); free(cf); free(bf);
    return 0;
}
