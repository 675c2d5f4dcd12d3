// sabr_dev.h -- device-side data layout and arithmetic for gfx950.
//
// Implied volatilities of static SABR (Section 2.1: eqs. "haganf",
// "sigma-SABR", "vola_SABR") and dynamic SABR (Section 2.2: eq.
// "vola_SABRd" with case I closed forms, eq. "exact-integral-expressions",
// or case II quadrature of eq. "integrales_SABRd"), the cost functions of
// Section 3, and Philox4x32-10 for the annealing and path draws.
//
// Precision policy: `R` is the bulk type (float or double).  In float mode
// the near-the-money ratio x(z)/z is summed in double from its Legendre
// series, the case I integrals switch to their Taylor series below a rate *
// maturity of 2, and every objective sum is accumulated in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sabr {

constexpr int kMaxPar = 10;
constexpr int kWG = 256;            // threads per annealing workgroup (4 waves)
constexpr int kMaxReaders = 8;      // workgroups that read a wide request's candidates (kWG each)
constexpr float kLn2f = 0.693147180559945309f;
constexpr double kLn2 = 0.693147180559945309417232121458;
constexpr double kZIsland = 0.05;   // |z| below which x(z)/z comes from its series

enum { MODEL_STATIC = 0, MODEL_DYN_I = 1, MODEL_DYN_II = 2 };
enum { F_HAGAN = 0, F_OBLOJ = 1, F_EXPANSION = 2 };
enum { W_ABSOLUTE = 0, W_RELATIVE = 1 };

// ---------------------------------------------------------------------------
// Packed problem description (device memory), one per calibration request.
// ---------------------------------------------------------------------------
struct ReqDesc {
    int32_t model, formula, weighting, beta_free;
    int32_t n_par, n_mat, n_pts;
    int32_t pt_off;       // first point in the batch point arrays
    int32_t mat_off;      // first maturity in the batch maturity arrays
    int32_t n_chains, n_iters, chain_len, n_levels;
    int32_t sched_off;    // first level in the schedule arrays
    int32_t wg_first, n_wg;   // workgroups of this request in the launch
    int32_t cand_off;     // first candidate slot (2 * n_wg slots)
    int32_t polish;
    int32_t rsplit;       // row split of a lane group: 0 rounds of one row per lane, else a fixed split dividing the lane count
    int32_t spin_limit;   // polls of a level-end slot before the wait gives up
    uint32_t key0, key1;
    double beta;
    double T0;            // <= 0: f(x0)
    double t_max;         // largest maturity (case II feasibility)
    double lb[kMaxPar], ub[kMaxPar], x0[kMaxPar];
};

// Point data of all requests of a batch (structure of arrays, double).
struct PointsD {
    const double *lfk;     // ln(f/K)
    const double *lkf;     // ln(K f)
    const double *P1;      // beta fixed: alpha-free leading factor
    const double *Z;       // beta fixed: z = (nu/alpha) * Z
    const double *Q1;      // beta fixed: (K f)^(-(1-beta)/2)
    const double *Q2;      // beta fixed: (K f)^(-(1-beta))
    const double *target;  // market value
    const double *sw;      // square root of the weight (1 or 1/target)
    const int32_t *row;    // maturity index of the point (global)
};
struct MatsD {
    const double *T;
    const double *lnf;     // ln f
    const double *F1;      // beta fixed: f^(1-beta)
    const int32_t *offs;   // global point offsets, n_mat + 1 per request (stored per request)
};

// Annealing chain state in device memory (between launches, for results).
struct ChainOut {
    double bf;
    double bx[kMaxPar];
};

// Level-end candidate of one workgroup: f, chain and x as 32-bit words, each
// stored in the low half of a 64-bit word whose high half is the exchange
// round + 1.  A 64-bit atomic access is indivisible, so a reader that sees the
// round in every word has the whole candidate of that round, with no fence.
constexpr int kCandWords = 3 + 2 * kMaxPar;
struct alignas(64) Cand {
    uint64_t w[kCandWords];
};

// ---------------------------------------------------------------------------
// Philox4x32-10, from its published definition (Salmon et al., SC'11).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Annealing uniform: (w + 1/2) 2^-32, exact in double.
__device__ __forceinline__ double unit_u32(uint32_t w) {
    return ((double)w + 0.5) * 2.3283064365386962890625e-10;
}
// Path uniform: top 24 bits, (w>>8 + 1/2) 2^-24, exact in float and double.
__device__ __forceinline__ float unit_u24f(uint32_t w) {
    return ((float)(w >> 8) + 0.5f) * 5.9604644775390625e-8f;
}
__device__ __forceinline__ double unit_u24d(uint32_t w) {
    return ((double)(w >> 8) + 0.5) * 5.9604644775390625e-8;
}

// ---------------------------------------------------------------------------
// x(z)/z from d x/d z = (1 - 2 rho z + z^2)^(-1/2): the Legendre generating
// function gives x(z)/z = sum_n P_n(rho) z^n / (n+1).  Used for |z| < 0.05,
// where the log form of eq. "equis" cancels.  NT terms, double.
// ---------------------------------------------------------------------------
template <int NT>
__device__ __forceinline__ double x_over_z_series(double z, double rho) {
    // q_n = P_n(rho) z^n by the Legendre recurrence in the variables rho z and
    // z^2: q_(n+1) = (2n+1)/(n+1) (rho z) q_n - n/(n+1) z^2 q_(n-1).
    const double t = rho * z, u = z * z;
    double qm = 1.0, q = t;
    double s = fma(0.5, t, 1.0);
#pragma unroll
    for (int n = 1; n < NT - 1; ++n) {
        const double qn = fma((double)(2 * n + 1) / (double)(n + 1) * t, q, -(double)n / (double)(n + 1) * u * qm);
        s = fma(1.0 / (double)(n + 2), qn, s);
        qm = q;
        q = qn;
    }
    return s;
}

// Coefficients c_n = P_n(rho) / (n + 1) of the same series, for evaluating it
// at many z with one rho (Horner in z), in the precision T.
template <typename T, int NT>
struct XzSeries {
    T c[NT];
    __device__ __forceinline__ void init(T rho) {
        T pm = (T)1, p = rho;
        c[0] = (T)1;
        c[1] = (T)0.5 * rho;
#pragma unroll
        for (int n = 1; n < NT - 1; ++n) {
            const T pn = fma((T)(2 * n + 1) / (T)(n + 1) * rho, p, -(T)n / (T)(n + 1) * pm);
            c[n + 1] = pn * ((T)1 / (T)(n + 2));
            pm = p;
            p = pn;
        }
    }
    __device__ __forceinline__ T eval(T z) const {
        T s = c[NT - 1];
#pragma unroll
        for (int n = NT - 2; n >= 0; --n) s = fma(s, z, c[n]);
        return s;
    }
};

// z / x(z), float bulk.  With zr = z - rho and s = sqrt(1 - 2 rho z + z^2):
// x = ln(s + zr) - ln(1 - rho) for zr >= 0, and, rationalising with
// (s + zr)(s - zr) = 1 - rho^2, x = ln(1 + rho) - ln(s - zr) for zr < 0;
// both are sign(zr) (ln(s + |zr|) - ln(1 -/+ rho)).  lr1 = ln(1 - rho),
// lr2 = ln(1 + rho) are per-chain constants.
__device__ __forceinline__ float x_log_f32(float z, float rho, float lr1, float lr2) {
    const float zr = z - rho;
    const float s = __builtin_amdgcn_sqrtf(fmaf(z, z - 2.0f * rho, 1.0f));
    const float lg = __builtin_amdgcn_logf(s + fabsf(zr)) * kLn2f;
    const float xl = lg - (zr >= 0.0f ? lr1 : lr2);
    return zr >= 0.0f ? xl : -xl;
}
__device__ __forceinline__ float z_over_x_f32(float z, float rho, float lr1, float lr2) {
    if (fabsf(z) < (float)kZIsland) return (float)(1.0 / x_over_z_series<8>((double)z, (double)rho));
    return z * __builtin_amdgcn_rcpf(x_log_f32(z, rho, lr1, lr2));
}

__device__ __forceinline__ double z_over_x_f64(double z, double rho, double lr1, double lr2) {
    if (fabs(z) < kZIsland) return 1.0 / x_over_z_series<15>(z, rho);
    const double zr = z - rho;
    const double s = sqrt(fma(z, z - 2.0 * rho, 1.0));
    const double xl = log(s + fabs(zr)) - (zr >= 0.0 ? lr1 : lr2);
    const double x = zr >= 0.0 ? xl : -xl;
    return z / x;
}

// ---------------------------------------------------------------------------
// Precision traits.
// ---------------------------------------------------------------------------
template <typename R> struct M;
template <> struct M<float> {
    static __device__ __forceinline__ float ex(float v) { return __builtin_amdgcn_exp2f(v * 1.44269504088896341f); }
    static __device__ __forceinline__ float lg(float v) { return __builtin_amdgcn_logf(v) * kLn2f; }
    static __device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
    static __device__ __forceinline__ float zx(float z, float r, float l1, float l2) { return z_over_x_f32(z, r, l1, l2); }
    static __device__ __forceinline__ float em1(float v) { return expm1f(v); }
};
template <> struct M<double> {
    static __device__ __forceinline__ double ex(double v) { return exp(v); }
    static __device__ __forceinline__ double lg(double v) { return log(v); }
    static __device__ __forceinline__ double rcp(double v) { return 1.0 / v; }
    static __device__ __forceinline__ double zx(double z, double r, double l1, double l2) { return z_over_x_f64(z, r, l1, l2); }
    static __device__ __forceinline__ double em1(double v) { return expm1(v); }
};

// ---------------------------------------------------------------------------
// Case I functional integrals (eq. "el_fun_1"): {nu1^2, nu2^2, eta1, eta2^2}
// divided by {nu0^2, nu0^2, nu0 rho0, nu0^2 rho0^2}, as functions of
// y = 2 b T and x = (a + b) T.  Above the switch point the closed forms of
// eq. "exact-integral-expressions"; below it the Taylor series of the same
// integrals (Beta integrals of the expanded exponential), by Horner:
//   n1(y) = sum 6 (-y)^k/(k+3)!,  n2(y) = sum 6 (k+1)(-y)^k/(k+3)!,
//   e1(x) = sum 2 (-x)^k/(k+2)!,  e2(x) = sum 3 (-1)^k (2^(k+4)-8) x^k/(k+4)!.
// ---------------------------------------------------------------------------
template <typename R> struct CaseI;
template <> struct CaseI<double> {
    static constexpr double kSwitch = 1.0;
    static constexpr int kN1 = 22, kN2 = 22, kE1 = 22, kE2 = 22;
};
// Float: below the switch point 2 the truncation after 12 / 13 / 13 / 16
// terms stays below the float rounding of the sums (largest relative error
// 2.6e-7 / 2.8e-7 / 3.2e-7 / 9.7e-7 over [0, 2], the same as with more terms).
template <> struct CaseI<float> {
    static constexpr double kSwitch = 2.0;
    static constexpr int kN1 = 12, kN2 = 13, kE1 = 13, kE2 = 16;
};

__host__ __device__ constexpr double factorial(int n) {
    double f = 1.0;
    for (int m = 2; m <= n; ++m) f *= (double)m;
    return f;
}
__host__ __device__ constexpr double pow2(int n) {
    double p = 1.0;
    for (int m = 0; m < n; ++m) p *= 2.0;
    return p;
}

// sum_{k < NT} c(k) z^k.  Float: E(z^2) + z O(z^2), two Horner chains of
// half the depth that the hardware runs side by side.  Double: one Horner
// chain (the reference evaluation order of the double path).
template <typename R, int NT, typename C>
__device__ __forceinline__ R series_even_odd(R z, C c) {
    static_assert(NT >= 2, "at least two terms");
    if constexpr (sizeof(R) == 8) {
        R h = (R)c(NT - 1);
#pragma unroll
        for (int k = NT - 2; k >= 0; --k) h = h * z + (R)c(k);
        return h;
    } else {
        // even terms up to 2 JE, odd terms up to 2 JO + 1, each chain started
        // at its top coefficient
        constexpr int JE = (NT - 1) / 2, JO = (NT - 2) / 2;
        const R u = z * z;
        R e = (R)c(2 * JE), o = (R)c(2 * JO + 1);
#pragma unroll
        for (int j = JE - 1; j >= 0; --j) e = e * u + (R)c(2 * j);
#pragma unroll
        for (int j = JO - 1; j >= 0; --j) o = o * u + (R)c(2 * j + 1);
        return e + z * o;
    }
}

template <typename R>
__device__ __forceinline__ void case1_normalised(R y, R x, R &n1, R &n2, R &e1, R &e2) {
    if (fabs((double)y) < CaseI<R>::kSwitch) {
        // c_k = 6/(k+3)! and 6(k+1)/(k+3)!
        n1 = series_even_odd<R, CaseI<R>::kN1>(-y, [](int k) { return 6.0 / factorial(k + 3); });
        n2 = series_even_odd<R, CaseI<R>::kN2>(-y, [](int k) { return 6.0 * (k + 1) / factorial(k + 3); });
    } else {
        const R ey = M<R>::ex(-y);
        const R c = (R)6 * M<R>::rcp(y * y * y);
        n1 = c * ((y * y * (R)0.5 - y + (R)1) - ey);
        n2 = c * ((R)2 * (ey - (R)1) + y * (ey + (R)1));
    }
    if (fabs((double)x) < CaseI<R>::kSwitch) {
        // c_k = 2/(k+2)! and 3 (2^(k+4) - 8)/(k+4)!
        e1 = series_even_odd<R, CaseI<R>::kE1>(-x, [](int k) { return 2.0 / factorial(k + 2); });
        e2 = series_even_odd<R, CaseI<R>::kE2>(-x, [](int k) { return 3.0 * (pow2(k + 4) - 8.0) / factorial(k + 4); });
    } else {
        const R ex = M<R>::ex(-x);
        const R ix2 = M<R>::rcp(x * x);
        e1 = (R)2 * ix2 * (ex - ((R)1 - x));
        e2 = (R)3 * ix2 * ix2 * (ex * ex - (R)8 * ex + ((R)7 + (R)2 * x * (x - (R)3)));
    }
}

// Case II functional integrals by composite Gauss-Legendre quadrature of
// eq. "integrales_SABRd".  I(s) = int_0^s nu rho du is carried panel by
// panel; eta2^2 uses int_0^T int_0^t g(s) ds dt = int_0^T (T - s) g(s) ds.
// Nodes of the 8-point rule on [-1, 1].
__device__ __forceinline__ double gl8_node(int i) {
    const double x[4] = {0.1834346424956498049394761, 0.5255324099163289858177390,
                         0.7966664774136267395915539, 0.9602898564975362316835609};
    return i < 4 ? -x[3 - i] : x[i - 4];
}
__device__ __forceinline__ double gl8_weight(int i) {
    const double w[4] = {0.3626837833783619829651504, 0.3137066458778872873379622,
                         0.2223810344533744705443560, 0.1012285362903762591525314};
    return i < 4 ? w[3 - i] : w[i - 4];
}

struct FnII {
    double rho0, nu0, a, b, drho, dnu, qrho, qnu;
    __device__ __forceinline__ double rho(double t) const { return fma(qrho, t, rho0) * exp(-a * t) + drho; }
    __device__ __forceinline__ double nu(double t) const { return fma(qnu, t, nu0) * exp(-b * t) + dnu; }
};

// Integral of nu*rho over [lo, hi] with the 8-point rule.
__device__ __forceinline__ double gl8_nurho(const FnII &p, double lo, double hi) {
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double t = fma(h, gl8_node(i), c);
        s = fma(gl8_weight(i), p.nu(t) * p.rho(t), s);
    }
    return s * h;
}

// Panels: n_panel equal panels on [0, T]; each outer node s needs I(s),
// built as I(panel start) + integral over [panel start, s] (8-point rule).
__device__ inline void case2_integrals(const FnII &p, double T, int n_panel, double out[4]) {
    const double hp = T / n_panel;
    double s1 = 0.0, s2 = 0.0, s3 = 0.0, s4 = 0.0, Ist = 0.0;
    for (int k = 0; k < n_panel; ++k) {
        const double lo = k * hp, hi = lo + hp;
        const double c = 0.5 * (lo + hi), h = 0.5 * hp;
        for (int i = 0; i < 8; ++i) {
            const double t = fma(h, gl8_node(i), c);
            const double w = gl8_weight(i) * h;
            const double nu = p.nu(t), rho = p.rho(t);
            const double Tt = T - t;
            s1 = fma(w, Tt * Tt * nu * nu, s1);
            s2 = fma(w, Tt * t * nu * nu, s2);
            s3 = fma(w, Tt * nu * rho, s3);
            const double I = Ist + gl8_nurho(p, lo, t);
            s4 = fma(w, Tt * I * I, s4);
        }
        Ist += gl8_nurho(p, lo, hi);
    }
    const double iT = 1.0 / T;
    out[0] = 3.0 * iT * iT * iT * s1;
    out[1] = 6.0 * iT * iT * iT * s2;
    out[2] = 2.0 * iT * iT * s3;
    out[3] = 12.0 * iT * iT * iT * iT * s4;
}

// Case II feasibility on (0, t_max]: each function is (c0 + c1 t) e^(-k t) + d,
// whose extrema lie at the ends or at t* = 1/k - c0/c1 (the derivative
// e^(-k t) (c1 - k (c0 + c1 t)) vanishes there for either sign of k, so
// growing exponentials are checked as well as decaying ones).
__device__ __forceinline__ void fn_range(double c0, double c1, double k, double d, double tmax,
                                         double &lo, double &hi) {
    const double v0 = c0 + d;
    const double v1 = fma(c1, tmax, c0) * exp(-k * tmax) + d;
    lo = fmin(v0, v1);
    hi = fmax(v0, v1);
    if (k != 0.0 && c1 != 0.0) {
        const double ts = 1.0 / k - c0 / c1;
        if (ts > 0.0 && ts < tmax) {
            const double v = fma(c1, ts, c0) * exp(-k * ts) + d;
            lo = fmin(lo, v);
            hi = fmax(hi, v);
        }
    }
}
__device__ __forceinline__ bool case2_feasible(const double *x, double tmax) {
    double rlo, rhi, nlo, nhi;
    fn_range(x[1], x[7], x[3], x[5], tmax, rlo, rhi);
    fn_range(x[2], x[8], x[4], x[6], tmax, nlo, nhi);
    return rlo >= -1.0 && rhi <= 1.0 && nlo > 0.0;
}

}  // namespace sabr
