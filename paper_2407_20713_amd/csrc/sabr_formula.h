// sabr_formula.h -- model implied volatilities and the market-fit objective
// on one parameter vector, evaluated by one lane over a market grid staged in
// LDS (Sections 2 and 3).
#pragma once
#include "sabr_dev.h"

namespace sabr {

// LDS point record (one per strike) and row record (one per maturity).
template <typename R>
struct alignas(16) Pt {
    R Z, PZW, Q1, Q2;     // beta fixed: z factor, |P1 Z| sqrt(weight), (Kf)^-(1-b)/2, (Kf)^-(1-b)
    R P1, lfk, lkf, T;    // leading factor, ln(f/K), ln(Kf), maturity
    R tsw, sw;            // market value times sqrt(weight), sqrt(weight)
};
template <typename R>
struct alignas(16) Row {
    R T, lnf, F1, pad;    // maturity, ln f, f^(1-beta) (beta fixed)
    int32_t p0, p1, q0, q1;
    int32_t spare[4];     // 48 bytes in float: lanes reading consecutive rows at once meet fewer LDS banks
};
// The point records are followed by kPtPad spare records, so that the point
// loops can read ahead past a row's end (the values read there are unused).
constexpr int kPtPad = 8;
template <typename R>
__host__ __device__ constexpr size_t pts_bytes(int n_pts) {
    return sizeof(Pt<R>) * (size_t)(n_pts + kPtPad);
}

template <int MODEL>
constexpr int base_npar() { return MODEL == MODEL_STATIC ? 3 : (MODEL == MODEL_DYN_I ? 5 : 9); }

// Grid normalisation of one point (double): ln(f/K), ln(Kf) and, for a fixed
// beta, the alpha-free factors of eqs. "haganf" / "sigma-SABR":
// Hagan: P1 = 1 / ((Kf)^((1-b)/2) den), Z = (Kf)^((1-b)/2) ln(f/K);
// Oblój: z = (nu/alpha) f^(1-b) l / g(u), leading factor alpha g(u) / f^(1-b),
// g(u) = u / (1 - e^-u), u = (1-b) l; den = 1 + (1-b)^2 l^2/24 + (1-b)^4 l^4/1920.
__device__ inline void normalise_point(double k, double f, double beta, int formula, int weighting, double t,
                                       double &lfk, double &lkf, double &P1, double &Z, double &Q1, double &Q2,
                                       double &sw) {
    const double omb = 1.0 - beta;
    const double l = log(f / k);
    const double lk = log(k * f);
    const double kf = exp(0.5 * omb * lk);
    const double l2 = l * l;
    const double den = 1.0 + omb * omb / 24.0 * l2 + omb * omb * omb * omb / 1920.0 * l2 * l2;
    lfk = l;
    lkf = lk;
    Q1 = 1.0 / kf;
    Q2 = 1.0 / (kf * kf);
    if (formula == F_OBLOJ) {
        const double F1 = exp(omb * log(f));
        const double u = omb * l;
        const double g = (u == 0.0) ? 1.0 : u / (-expm1(-u));
        P1 = g / (F1 * den);
        Z = F1 * l / g;
    } else {
        P1 = 1.0 / (kf * den);
        Z = kf * l;
    }
    sw = (weighting == W_RELATIVE) ? 1.0 / t : 1.0;
}

// Stage the points and rows of one request into LDS (all threads of the
// block take part; the caller synchronises afterwards).  With row_pad, a row
// of even length is followed by one spare record, so that the rows' starts
// fall on different LDS banks (lanes reading different rows at once then
// conflict less: a 48-byte record is 12 banks wide, and a stride of an odd
// number of records spreads 8 rows over distinct bank groups); the rows' p0
// and p1 index the padded records.
template <typename R>
__device__ inline void stage_grid(const ReqDesc &rq, const PointsD &P, const MatsD &Mt,
                                  Pt<R> *pts, Row<R> *rows, bool row_pad = false) {
    for (int i = threadIdx.x; i < rq.n_mat; i += blockDim.x) {
        const int g = rq.mat_off + i;
        int shift = 0;
        if (row_pad)
            for (int k = 0; k < i; ++k)
                shift += ((Mt.offs[rq.mat_off + k + 1] - Mt.offs[rq.mat_off + k]) & 1) == 0;
        Row<R> r;
        r.T = (R)Mt.T[g];
        r.lnf = (R)Mt.lnf[g];
        r.F1 = (R)Mt.F1[g];
        r.pad = (R)0;
        r.p0 = Mt.offs[g] - rq.pt_off + shift;
        r.p1 = Mt.offs[g + 1] - rq.pt_off + shift;
        r.q0 = r.q1 = 0;
        rows[i] = r;
    }
    if (row_pad) __syncthreads();   // the points read their rows' padded starts
    for (int j = threadIdx.x; j < rq.n_pts; j += blockDim.x) {
        const int g = rq.pt_off + j;
        int slot = j;
        if (row_pad) {
            const int r = P.row[g] - rq.mat_off;
            slot = j + rows[r].p0 - (Mt.offs[rq.mat_off + r] - rq.pt_off);
        }
        Pt<R> p;
        p.P1 = (R)P.P1[g];
        p.Z = (R)P.Z[g];
        p.PZW = (R)fabs(P.P1[g] * P.Z[g] * P.sw[g]);
        p.Q1 = (R)P.Q1[g];
        p.Q2 = (R)P.Q2[g];
        p.lfk = (R)P.lfk[g];
        p.lkf = (R)P.lkf[g];
        p.T = (R)Mt.T[P.row[g]];
        p.sw = (R)P.sw[g];
        p.tsw = (R)(P.target[g] * P.sw[g]);
        pts[slot] = p;
    }
}

// Row block of the expansion and of the dynamic formula:
// sigma = inv_w (c0 + L (A1 + A2 L)) with L = ln(K/f), c0 = 1 + B T.
template <typename R>
struct Quad {
    R inv_w, A1, A2, c0;
};

// eq. "vola_SABR": omega = f^(1-beta)/alpha.
template <typename R>
__device__ __forceinline__ Quad<R> expansion_block(R F1, R T, R al, R beta, R rho, R nu) {
    const R omb = (R)1 - beta;
    const R w = F1 / al;
    const R rnw = rho * nu * w;
    const R c3 = (R)2 - (R)3 * rho * rho;
    Quad<R> q;
    q.inv_w = al / F1;
    q.A1 = (R)-0.5 * (omb - rnw);
    q.A2 = (omb * omb + (R)3 * (omb - rnw) + c3 * nu * nu * w * w) * (R)(1.0 / 12.0);
    const R B = omb * omb * (R)(1.0 / 24.0) * q.inv_w * q.inv_w + beta * rho * nu * (R)0.25 * q.inv_w
              + c3 * (R)(1.0 / 24.0) * nu * nu;
    q.c0 = fma(B, T, (R)1);
    return q;
}

// eq. "vola_SABRd" from the four integrals {nu1^2, nu2^2, eta1, eta2^2}.
template <typename R>
__device__ __forceinline__ Quad<R> dynamic_block(R F1, R T, R al, R beta, R n1sq, R n2sq, R e1, R e2sq) {
    const R omb = (R)1 - beta;
    Quad<R> q;
    R w;
    if constexpr (sizeof(R) == 4) {
        // float bulk: hardware reciprocals (1 ulp) instead of two divisions
        w = F1 * M<R>::rcp(al);
        q.inv_w = al * M<R>::rcp(F1);
    } else {
        w = F1 / al;
        q.inv_w = al / F1;
    }
    q.A1 = (beta - (R)1) * (R)0.5 + e1 * w * (R)0.5;
    q.A2 = omb * omb * (R)(1.0 / 12.0) + (omb - e1 * w) * (R)0.25
         + ((R)4 * n1sq + (R)3 * (e2sq - (R)3 * e1 * e1)) * (R)(1.0 / 24.0) * w * w;
    const R B = q.inv_w * q.inv_w * (omb * omb * (R)(1.0 / 24.0) + w * beta * e1 * (R)0.25
                                     + ((R)2 * n2sq - (R)3 * e2sq) * (R)(1.0 / 24.0) * w * w);
    q.c0 = fma(B, T, (R)1);
    return q;
}

// Model implied vol of one parameter vector, split into the part that depends
// on the vector alone (init), on the maturity row (row) and on the strike
// (point), so that a lane can evaluate a whole grid (objective) or a single
// point (polish).
template <int MODEL, int FORMULA, typename R, bool BFREE, typename P = double>
struct ModelEval {
    R al, rh, nu, beta, omb;
    R noa, c1a2, c2rna, c3n2, lr1, lr2, d1, d2;   // z-form static formulas
    R an, lb1, lb2, omr2;                         // float hot loop: nu / ln 2, log2(1 -/+ rho), 1 - rho^2
    R F1;                                         // f^(1-beta) of the current row
    Quad<R> q;                                    // expansion / dynamic row block
    const P *y;   // parameter vector (double, or float in the float annealing)

    // Returns false for a case II vector outside rho(t) in [-1,1], nu(t) > 0.
    __device__ __forceinline__ bool init(const P *y_, double beta_fixed, double t_max) {
        constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
        y = y_;
        const double beta_d = BFREE ? (double)y[NP - 1] : beta_fixed;
        al = (R)y[0];
        rh = (R)y[1];
        nu = (R)y[2];
        beta = (R)beta_d;
        omb = (R)(1.0 - beta_d);
        if constexpr (MODEL == MODEL_STATIC && FORMULA != F_EXPANSION) {
            if constexpr (sizeof(R) == 4)
                noa = nu * M<R>::rcp(al);   // hardware reciprocal (1 ulp) in the float bulk
            else
                noa = nu / al;
            c1a2 = omb * omb * (R)(1.0 / 24.0) * al * al;
            c2rna = beta * (R)0.25 * rh * nu * al;
            c3n2 = ((R)2 - (R)3 * rh * rh) * (R)(1.0 / 24.0) * nu * nu;
            if constexpr (sizeof(R) == 4) {
                lb1 = __builtin_amdgcn_logf(1.0f - rh);
                lb2 = __builtin_amdgcn_logf(1.0f + rh);
                lr1 = lb1 * kLn2f;
                lr2 = lb2 * kLn2f;
                an = nu * 1.44269504088896341f;   // al noa = nu
                omr2 = (1.0f - rh) * (1.0f + rh);
            } else {
                lr1 = M<R>::lg((R)1 - rh);
                lr2 = M<R>::lg((R)1 + rh);
            }
            d1 = omb * omb * (R)(1.0 / 24.0);
            d2 = d1 * d1 * (R)(576.0 / 1920.0);
        }
        if constexpr (MODEL == MODEL_DYN_II) {
            if constexpr (sizeof(P) == 8) {
                return case2_feasible(y, t_max);
            } else {
                double yd[9];
#pragma unroll
                for (int k = 0; k < 9; ++k) yd[k] = (double)y[k];
                return case2_feasible(yd, t_max);
            }
        }
        return true;
    }

    __device__ __forceinline__ void row(const Row<R> &rw) {
        if constexpr (MODEL == MODEL_STATIC && FORMULA != F_EXPANSION) {
            F1 = rw.F1;
            if (BFREE && FORMULA == F_OBLOJ) F1 = M<R>::ex(omb * rw.lnf);
        } else {
            F1 = BFREE ? M<R>::ex(omb * rw.lnf) : rw.F1;
            if constexpr (MODEL == MODEL_STATIC) {
                q = expansion_block<R>(F1, rw.T, al, beta, rh, nu);
            } else if constexpr (MODEL == MODEL_DYN_I) {
                const R a = (R)y[3], b = (R)y[4];
                R n1, n2, e1, e2;
                case1_normalised<R>((R)2 * b * rw.T, (a + b) * rw.T, n1, n2, e1, e2);
                const R nr = nu * rh;
                q = dynamic_block<R>(F1, rw.T, al, beta, nu * nu * n1, nu * nu * n2, nr * e1, nr * nr * e2);
            } else {
                FnII fp{y[1], y[2], y[3], y[4], y[5], y[6], y[7], y[8]};
                const double Td = (double)rw.T;
                const double kmax = fmax(fmax(fabs(y[3]), fabs(y[4])), 1.0);   // growing rates too
                int np = (int)ceil(Td * kmax);
                np = np < 1 ? 1 : (np > 64 ? 64 : np);
                double ints[4];
                case2_integrals(fp, Td, np, ints);
                q = dynamic_block<R>(F1, rw.T, al, beta, (R)ints[0], (R)ints[1], (R)ints[2], (R)ints[3]);
            }
            if constexpr (sizeof(R) == 4) {
                // float: inv_w folded into the row's coefficients (one
                // multiplication per row instead of one per point)
                q.A1 *= q.inv_w;
                q.A2 *= q.inv_w;
                q.c0 *= q.inv_w;
            }
        }
    }

    // z / x(z) for |z| < kZIsland (float bulk), from the series where the log
    // form cancels: x(z)/z = 1 + z (c1 + z (c2 + z (c3 + z (c4 + z c5)))),
    // c_n = P_n(rho) / (n + 1).  |z| < 0.05 and |P_n(rho)| <= 1, so the six
    // terms leave a truncation below 0.05^6 / 7 = 2.3e-9.  The outer two terms
    // are formed in double; the inner part c2 + z (...), at most 0.05^2 of the
    // sum, in float (its rounding then counts below 1e-10 of the sum).  z = 0
    // (the strike at the forward) is the limit 1.
    __device__ __forceinline__ float zx_near(float z) const {
        if (z == 0.0f) return 1.0f;
        const float p2 = fmaf(1.5f * rh, rh, -0.5f);
        const float p3 = fmaf(5.0f / 3.0f * rh, p2, -2.0f / 3.0f * rh);
        const float p4 = fmaf(7.0f / 4.0f * rh, p3, -0.75f * p2);
        const float p5 = fmaf(9.0f / 5.0f * rh, p4, -0.8f * p3);
        const float inner = fmaf(z, fmaf(z, fmaf(z, p5 * (1.0f / 6.0f), p4 * 0.2f), p3 * 0.25f), p2 * (1.0f / 3.0f));
        const double zd = (double)z;
        const double s = fma(zd, fma(zd, (double)inner, 0.5 * (double)y[1]), 1.0);
        return __builtin_amdgcn_rcpf((float)s);
    }

    __device__ __forceinline__ R point(const Pt<R> &p) const {
        if constexpr (MODEL == MODEL_STATIC && FORMULA != F_EXPANSION) {
            R P1, Z, Q1, Q2;
            if constexpr (!BFREE) {
                P1 = p.P1; Z = p.Z; Q1 = p.Q1; Q2 = p.Q2;
            } else {
                const R kf = M<R>::ex((R)0.5 * omb * p.lkf);
                Q1 = M<R>::rcp(kf);
                Q2 = Q1 * Q1;
                const R l2 = p.lfk * p.lfk;
                const R den = fma(l2, fma(d2, l2, d1), (R)1);
                if (FORMULA == F_HAGAN) {
                    P1 = Q1 * M<R>::rcp(den);
                    Z = kf * p.lfk;
                } else {
                    const R u = omb * p.lfk;
                    const R g = (u == (R)0) ? (R)1 : u / (-M<R>::em1(-u));
                    P1 = g * M<R>::rcp(F1 * den);
                    Z = F1 * p.lfk / g;
                }
            }
            const R z = noa * Z;
            R zx;
            if constexpr (sizeof(R) == 4) {
                zx = (fabsf(z) < (float)kZIsland) ? zx_near(z) : z * __builtin_amdgcn_rcpf(x_log_f32(z, rh, lr1, lr2));
            } else {
                zx = M<R>::zx(z, rh, lr1, lr2);
            }
            const R corr = fma(fma(c1a2, Q2, fma(c2rna, Q1, c3n2)), p.T, (R)1);
            return al * P1 * zx * corr;
        } else {
            const R L = -p.lfk;
            if constexpr (sizeof(R) == 4) return fma(L, fma(q.A2, L, q.A1), q.c0);   // inv_w folded in
            return q.inv_w * fma(L, fma(q.A2, L, q.A1), q.c0);
        }
    }
};

template <typename R>
__device__ __forceinline__ bool vol_ok(R sig) { return sig > (R)0 && sig < (R)__builtin_inff(); }

// Objective of one parameter vector y (double) over the staged grid:
// sum over points of ((target - model) * sw)^2, accumulated in double.
// A model vol that is not finite and positive, or an infeasible case II
// vector, gives +inf.  WRITE stores the model vols to out[0..n_pts).
// With LPC > 1 lanes per parameter vector, lane `sub` returns a partial sum.
// The static z-form loop splits the points of every row over the lanes; the
// other formulas give each lane whole rows where they can, so that a row's
// integrals are computed by fewer lanes than its points (rsplit 0), or split
// the rows over `rsplit` lanes and the points of each row over the other
// LPC / rsplit lanes.
template <int MODEL, int FORMULA, typename R, bool BFREE, bool WRITE, int LPC = 1, typename P = double>
__device__ double objective(const P *y, const Pt<R> *pts, const Row<R> *rows, int n_mat,
                            double beta_fixed, double t_max, double *out, int sub = 0, int rsplit = 1,
                            Row<R> r0 = Row<R>{}, bool have_r0 = false) {
    ModelEval<MODEL, FORMULA, R, BFREE, P> ev;
    if (!ev.init(y, beta_fixed, t_max)) return __builtin_inf();
    bool bad = false;
    // The hot loop folds nu / ln 2 into the maturity factor and divides by
    // nu for the island bound, so a vanishing nu (the box allows nu = 0, where
    // z / x(z) = 1 and the vol has its finite limit) takes the generic loop.
    if constexpr (MODEL == MODEL_STATIC && FORMULA != F_EXPANSION && !BFREE && sizeof(R) == 4 && !WRITE)
    if (ev.nu >= 1e-20f) {
        // float hot loop of the static z-form formulas, two points per step so
        // that their dependency chains interleave.  With zr = z - rho and
        // q = sqrt(zr^2 + 1 - rho^2) (= sqrt(1 - 2 rho z + z^2)), x(z) / ln 2 is
        // log2(q + zr) - log2(1 - rho) for zr >= 0 and log2(1 + rho) -
        // log2(q - zr) for zr < 0 (rationalised as in x_log_f32), so the vol is
        // (P1 Z) (nu / ln 2) corr / (x / ln 2); near the money, where that form
        // cancels, al P1 corr (z / x) from the series.  The maturity factor
        // corr = 1 + T (c1a2 Q2 + c2rna Q1 + c3n2) takes its T from the row;
        // its coefficients carry the factor nu / ln 2.  Both branches of x / ln 2
        // are +-(L - lb) with lb = log2(1 - rho) or log2(1 + rho), and x has
        // the sign of z, that is of Z, as P1 Z does; so (P1 Z) / x =
        // |P1 Z| / |L - lb| and the sign never has to be applied.  The
        // residual sqrt(w) (target - vol) is one fma,
        // tsw - (|P1 Z| sqrt(w) corr) / |L - lb|, with |P1 Z| sqrt(w) staged
        // per point; residuals in float, their squares summed in double (the
        // sums that decide the Metropolis test).
        // A vol that is not finite and positive makes the objective +inf.
        // Its sign is corr's: the other factors are |P1 Z| sqrt(w) and
        // 1 / |L - lb| (in the island P1, sqrt(w) and z / x, all positive),
        // so the check is on the smallest corr, and a non-finite vol makes
        // the sum infinite or NaN.  The smallest
        // corr is tracked on the bit patterns as signed integers: for
        // non-negative floats that order is the float order, and every float
        // with its sign bit set (negative, -0, negative NaN) compares below
        // +0, so `> 0` holds exactly when each corr is a positive number,
        // +inf or a NaN with the sign bit clear, and those last two make the
        // sum infinite or NaN.  (An integer minimum needs no NaN
        // canonicalisation.)
        const float noa = ev.noa, rh = ev.rh, lb1 = ev.lb1, lb2 = ev.lb2, omr2 = ev.omr2;
        // near the money: |z| = noa |Z| < kZIsland
        // al / nu, from one hardware reciprocal: the island bound and the
        // island's scale al / an = (al / nu) ln 2 both derive from it
        const float aln = ev.al * __builtin_amdgcn_rcpf(ev.nu);
        const float zthr = (float)kZIsland * aln;
        const float iscale = aln * 0.693147180559945309f;
        float k0 = 0.0f, k1 = 0.0f, k2 = 0.0f;
        double acc_a = 0.0, acc_b = 0.0;
        int cmin = 0x7fffffff;
        auto resid = [&](const Pt<R> &p, float &e, float &corr, bool &isl) {
            const float zr = fmaf(noa, p.Z, -rh);
            const float q = __builtin_amdgcn_sqrtf(fmaf(zr, zr, omr2));
            const float L = __builtin_amdgcn_logf(q + fabsf(zr));
            const float d = L - (zr >= 0.0f ? lb1 : lb2);
            corr = fmaf(k1, p.Q2, fmaf(k2, p.Q1, k0));
            e = fmaf(-(p.PZW * corr), __builtin_amdgcn_rcpf(fabsf(d)), p.tsw);
            isl = fabsf(p.Z) < zthr;
        };
        auto island = [&](const Pt<R> &p, float corr) {
            const float sg = iscale * p.P1 * corr * ev.zx_near(noa * p.Z);
            return fmaf(-sg, p.sw, p.tsw);
        };
        auto pair = [&](const Pt<R> &pa, const Pt<R> &pb) {
            float ea, eb, ca, cb;
            bool ia, ib;
            resid(pa, ea, ca, ia);
            resid(pb, eb, cb, ib);
            if (__builtin_expect(ia || ib, 0)) {
                if (ia) ea = island(pa, ca);
                if (ib) eb = island(pb, cb);
            }
            cmin = min(min(cmin, __float_as_int(ca)), __float_as_int(cb));
            acc_a = fma((double)ea, (double)ea, acc_a);
            acc_b = fma((double)eb, (double)eb, acc_b);
        };
        auto single = [&](const Pt<R> &p) {
            float e, c;
            bool is;
            resid(p, e, c, is);
            if (is) e = island(p, c);
            cmin = min(cmin, __float_as_int(c));
            acc_a = fma((double)e, (double)e, acc_a);
        };
        for (int i = 0; i < n_mat; ++i) {
            const Row<R> rw = (i == 0 && have_r0) ? r0 : rows[i];
            int j = rw.p0 + sub;
            if (j >= rw.p1) continue;
            k0 = ev.an * fmaf(ev.c3n2, rw.T, 1.0f);
            k1 = ev.an * (ev.c1a2 * rw.T);
            k2 = ev.an * (ev.c2rna * rw.T);
            // two pairs per step, each pair's records loaded while the other
            // is computed (two register sets, no copies); reads past the
            // row's end land in the next row or the spare records, unused.
            // The steps every lane of the group can take (the row is the same
            // for the whole wave) run under one wave-wide count; the last
            // one to four points of a lane follow.
            static_assert(LPC <= 2, "the read-ahead stays within the spare point records");
            const int nq = __builtin_amdgcn_readfirstlane(((rw.p1 - rw.p0) / LPC) / 4);
            const Pt<R> *pp = pts + j;
            Pt<R> a0 = pp[0], b0 = pp[LPC];
            for (int q = 0; q < nq; ++q, pp += 4 * LPC) {
                const Pt<R> a1 = pp[2 * LPC], b1 = pp[3 * LPC];
                pair(a0, b0);
                a0 = pp[4 * LPC];
                b0 = pp[5 * LPC];
                pair(a1, b1);
            }
            j += 4 * LPC * nq;
            if (j + LPC < rw.p1) {
                pair(a0, b0);
                if (j + 3 * LPC < rw.p1)
                    pair(pp[2 * LPC], pp[3 * LPC]);
                else if (j + 2 * LPC < rw.p1)
                    single(pp[2 * LPC]);
            } else if (j < rw.p1) {
                single(a0);
            }
        }
        const double acc = acc_a + acc_b;
        return (cmin > 0 && acc < __builtin_inf()) ? acc : __builtin_inf();
    }
    // float: points in pairs with their own partial sums (two independent
    // dependency chains), added once at the end; residuals in float, their
    // squares summed in double (so the sum hardly depends on how the points
    // are split over lanes); double: one sum in point order
    constexpr bool kTwo = sizeof(R) == 4;
    // float without model output: the smallest vol tracked on the bit patterns
    // as signed integers (every float with its sign bit set, and +0, compare
    // at or below 0; +inf and NaN make the sum infinite or NaN), one integer
    // minimum per point instead of two tests
    constexpr bool kIntMin = kTwo && !WRITE;
    constexpr bool kFour = kTwo && MODEL != MODEL_STATIC;
    int cmin = 0x7fffffff;
    double acc1 = 0.0, acc2 = 0.0;
    auto take = [&](const Pt<R> &p, R sig, double &acc) {
        if constexpr (kIntMin)
            cmin = min(cmin, __builtin_bit_cast(int, (float)sig));
        else
            bad |= !vol_ok(sig);
        const double e = (double)fma(-sig, p.sw, p.tsw);
        acc = fma(e, e, acc);
    };
    // points first, first + step, ... of row i; in float four at a time
    // where the model's row blocks leave the registers for it (the four
    // records read together, one LDS wait per four points), then in pairs,
    // then one
    auto row_points = [&](int i, int first, int step) {
        const Row<R> rw = rows[i];
        ev.row(rw);
        int j = rw.p0 + first;
        for (; kFour && j + 3 * step < rw.p1; j += 4 * step) {
            const Pt<R> pa = pts[j], pb = pts[j + step], pc = pts[j + 2 * step], pd = pts[j + 3 * step];
            const R sa = ev.point(pa), sb = ev.point(pb), sc = ev.point(pc), sd = ev.point(pd);
            take(pa, sa, acc1);
            take(pb, sb, acc2);
            take(pc, sc, acc1);
            take(pd, sd, acc2);
            if (WRITE) {
                out[j] = (double)sa;
                out[j + step] = (double)sb;
                out[j + 2 * step] = (double)sc;
                out[j + 3 * step] = (double)sd;
            }
        }
        auto pair = [&](int jj) {
            const Pt<R> pa = pts[jj], pb = pts[jj + step];
            const R sa = ev.point(pa), sb = ev.point(pb);
            take(pa, sa, acc1);
            take(pb, sb, acc2);
            if (WRITE) {
                out[jj] = (double)sa;
                out[jj + step] = (double)sb;
            }
        };
        if constexpr (kFour) {
            if (j + step < rw.p1) {   // at most one pair after the fours
                pair(j);
                j += 2 * step;
            }
        } else {
            for (; kTwo && j + step < rw.p1; j += 2 * step) pair(j);
        }
        for (; j < rw.p1; j += step) {
            const Pt<R> p = pts[j];
            const R sig = ev.point(p);
            take(p, sig, acc1);
            if (WRITE) out[j] = (double)sig;
        }
    };
    if (LPC == 1) {
        for (int i = 0; i < n_mat; ++i) row_points(i, 0, 1);
    } else if (rsplit > 0) {
        // fixed split: lane sub % rsplit takes rows sub % rsplit (mod rsplit),
        // the other LPC / rsplit lanes of the row split its points
        const int RS = rsplit, PS = LPC / rsplit;
        for (int i = sub % RS; i < n_mat; i += RS) row_points(i, sub / RS, PS);
    } else {
        // whole rounds of LPC rows, one row per lane with all its points; the
        // remaining rows (fewer than LPC) over the smallest power of two of
        // lanes that holds them, the other lanes of each such row splitting its
        // points.  Fewer row blocks and fewer points per lane than any fixed
        // split when the rows are not a multiple of the group size.
        int i0 = 0;
        for (; i0 + LPC <= n_mat; i0 += LPC) row_points(i0 + sub, 0, 1);
        const int rem = n_mat - i0;
        if (rem > 0) {
            int rs = 1;
            while (rs < rem) rs *= 2;
            if (sub % rs < rem) row_points(i0 + sub % rs, sub / rs, LPC / rs);
        }
    }
    if constexpr (kTwo) acc1 = acc1 + acc2;
    if constexpr (kIntMin) return (cmin > 0 && acc1 < __builtin_inf()) ? acc1 : __builtin_inf();
    return bad ? __builtin_inf() : acc1;
}

}  // namespace sabr
