// kernels_formula.hip -- grid normalisation, batch objective, persistent
// synchronous annealing and Levenberg-Marquardt polish (Sections 2, 3 and 5).
#include "sabr_formula.h"
#include "sabr_kernels.h"
#include "sabr_sa.h"

namespace sabr {

// ---------------------------------------------------------------------------
// Grid normalisation: per point ln(f/K), ln(Kf), and for a fixed beta the
// alpha-free factors of eqs. "haganf" / "sigma-SABR"; per maturity ln f and
// f^(1-beta).  Double precision, one thread per point / maturity.
// ---------------------------------------------------------------------------
__global__ void prepare_points_kernel(int n_pts, const double *K, const double *fwd_of_pt,
                                      const double *beta_of_pt, const int32_t *formula_of_pt,
                                      const int32_t *weighting_of_pt, const double *target,
                                      double *lfk, double *lkf, double *P1, double *Z, double *Q1,
                                      double *Q2, double *sw) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pts) return;
    normalise_point(K[j], fwd_of_pt[j], beta_of_pt[j], formula_of_pt[j], weighting_of_pt[j],
                    target ? target[j] : 0.0, lfk[j], lkf[j], P1[j], Z[j], Q1[j], Q2[j], sw[j]);
}

__global__ void prepare_mats_kernel(int n_mat, const double *fwd, const double *beta_of_mat,
                                    double *lnf, double *F1) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_mat) return;
    lnf[i] = log(fwd[i]);
    F1[i] = exp((1.0 - beta_of_mat[i]) * log(fwd[i]));
}

// ---------------------------------------------------------------------------
// Batch objective: lane = parameter vector, grid staged in LDS.
// ---------------------------------------------------------------------------
template <int MODEL, int FORMULA, typename R, bool BFREE>
__global__ void __launch_bounds__(256) objective_kernel(const ReqDesc *rqp, PointsD P, MatsD Mt,
                                                        const double *X, int64_t n_x, double *f,
                                                        double *model, int write_f) {
    extern __shared__ unsigned char smem[];
    const ReqDesc &rq = *rqp;
    Pt<R> *pts = reinterpret_cast<Pt<R> *>(smem);
    Row<R> *rows = reinterpret_cast<Row<R> *>(smem + pts_bytes<R>(rq.n_pts));
    stage_grid<R>(rq, P, Mt, pts, rows);
    __syncthreads();
    constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
    const int n_mat = rq.n_mat;
    const double beta = rq.beta, tmax = rq.t_max;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_x;
         i += (int64_t)gridDim.x * blockDim.x) {
        double y[NP];
#pragma unroll
        for (int k = 0; k < NP; ++k) y[k] = X[i * NP + k];
        double v;
        if (model)
            v = objective<MODEL, FORMULA, R, BFREE, true>(y, pts, rows, n_mat, beta, tmax,
                                                          model + i * rq.n_pts);
        else
            v = objective<MODEL, FORMULA, R, BFREE, false>(y, pts, rows, n_mat, beta, tmax, nullptr);
        if (write_f) f[i] = v;
    }
}

// ---------------------------------------------------------------------------
// Persistent synchronous annealing (Section 5, Technique I).  One lane is
// one Markov chain; the workgroups of a request exchange their best state
// at each level end; every chain restarts from the request's best.
// ---------------------------------------------------------------------------
template <int MODEL, int FORMULA, typename R, bool BFREE, int LPC>
__global__ void __launch_bounds__(kWG, 3) sa_kernel(const ReqDesc *reqs, const int32_t *wg_req,
                                                 PointsD P, MatsD Mt, const double *sched_g,
                                                 const double *sched_h, Cand *cands,
                                                 ChainOut *best_out, unsigned long long *accepts,
                                                 int32_t *err) {
    constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
    constexpr int NB = (NP + 1 + 3) / 4;   // Philox blocks per iteration
    extern __shared__ unsigned char smem[];
    const int req = wg_req[blockIdx.x];
    const ReqDesc &rq = reqs[req];
    ArgminSmem &am = *reinterpret_cast<ArgminSmem *>(smem);
    double *s_lb = reinterpret_cast<double *>(smem + sizeof(ArgminSmem));
    double *s_ub = s_lb + kMaxPar;
    Pt<R> *pts = reinterpret_cast<Pt<R> *>(smem + sizeof(ArgminSmem) + 2 * kMaxPar * sizeof(double));
    // wide lane groups take whole rows on different lanes at once: spare
    // records between the rows spread their starts over the LDS banks
    constexpr bool kRowPad = LPC > 2;
    Row<R> *rows = reinterpret_cast<Row<R> *>(reinterpret_cast<unsigned char *>(pts) +
                                              pts_bytes<R>(rq.n_pts + (kRowPad ? rq.n_mat : 0)));
    stage_grid<R>(rq, P, Mt, pts, rows, kRowPad);
    if (threadIdx.x < NP) {
        s_lb[threadIdx.x] = rq.lb[threadIdx.x];
        s_ub[threadIdx.x] = rq.ub[threadIdx.x];
    }
    __syncthreads();

    // LPC lanes share one chain: each takes every LPC-th strike and the
    // partial sums are combined across the lane group; the chain state and
    // its random words are the same on every lane of the group.
    const int wg_local = blockIdx.x - rq.wg_first;
    const int sub = threadIdx.x % LPC;
    const int chain = wg_local * (kWG / LPC) + threadIdx.x / LPC;
    const bool active = chain < rq.n_chains;
    const int n_mat = rq.n_mat, L = rq.chain_len, n_iters = rq.n_iters;
    const double beta = rq.beta, tmax = rq.t_max;
    const int rsplit = rq.rsplit;
    const uint32_t k0 = rq.key0, k1 = rq.key1;
    const Row<R> r0 = rows[0];   // the first row's record, kept in registers
    auto f_of = [&](const auto *v) {
        double part = objective<MODEL, FORMULA, R, BFREE, false, LPC>(v, pts, rows, n_mat, beta, tmax, nullptr, sub,
                                                                      rsplit, r0, true);
        return group_sum<LPC>(part);
    };

    double x[NP], bx[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) x[k] = bx[k] = rq.x0[k];
    double fx = f_of(x);
    const double T0 = rq.T0 > 0.0 ? rq.T0 : ((fx > 0.0 && fx < __builtin_inf()) ? fx : 1.0);
    double fb = fx;
    unsigned long long nacc = 0;
    int round = 0;

    for (int lev = 0; lev < rq.n_levels; ++lev) {
        const double g = sched_g[rq.sched_off + lev];
        const double h = sched_h[rq.sched_off + lev];
        const double Tk = T0 * g;
        const int t1 = min((lev + 1) * L, n_iters);
        if (active) sa_level<NP, NB, LPC, R>(chain, sub, lev * L, t1, k0, k1, h, Tk, s_lb, s_ub, x, fx, bx, fb, nacc, f_of);
        if (!request_argmin<NP>(fx, chain, active, x, am, rq, wg_local, round++, cands, err)) return;
        fx = am.bf;
#pragma unroll
        for (int k = 0; k < NP; ++k) x[k] = am.bx[k];
        __syncthreads();
    }
    // best-so-far over all chains of the request
    if (!request_argmin<NP>(fb, chain, active, bx, am, rq, wg_local, round++, cands, err)) return;
    // accepted moves: workgroup sum, one integer atomic per workgroup
    unsigned long long a = (active && sub == 0) ? nacc : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    __shared__ unsigned long long s_acc[kWG / 64];
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tot += s_acc[w];
        atomicAdd(&accepts[req], tot);
        if (wg_local == 0) {
            best_out[req].bf = am.bf;
            for (int k = 0; k < NP; ++k) best_out[req].bx[k] = am.bx[k];
        }
    }
}

template <int MODEL, int FORMULA, bool BFREE>
__global__ void __launch_bounds__(64) polish_kernel(const ReqDesc *reqs, const int32_t *req_ids,
                                                    PointsD P, MatsD Mt, ChainOut *best,
                                                    unsigned long long *evals) {
    constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
    extern __shared__ unsigned char smem[];
    const int req = req_ids[blockIdx.x];
    const ReqDesc &rq = reqs[req];
    Pt<double> *pts = reinterpret_cast<Pt<double> *>(smem);
    Row<double> *rows = reinterpret_cast<Row<double> *>(smem + pts_bytes<double>(rq.n_pts));
    int32_t *prow = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(rows) + sizeof(Row<double>) * rq.n_mat);
    stage_grid<double>(rq, P, Mt, pts, rows);
    __syncthreads();
    for (int i = 0; i < rq.n_mat; ++i)
        for (int j = rows[i].p0 + threadIdx.x; j < rows[i].p1; j += 64) prow[j] = i;
    __syncthreads();
    double x[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) x[k] = best[req].bx[k];
    unsigned long long ne = 0;
    const double fx = lm_polish<MODEL, FORMULA, BFREE>(x, pts, rows, prow, rq, &ne);
    if (threadIdx.x == 0) {
        if (fx <= best[req].bf || !(best[req].bf < __builtin_inf())) {
            best[req].bf = fx;
            for (int k = 0; k < NP; ++k) best[req].bx[k] = x[k];
        }
        evals[req] = ne;
    }
}

// ---------------------------------------------------------------------------
// Template instantiation tables.
// ---------------------------------------------------------------------------
#define SABR_FORMULA_VARIANTS(X)                                  \
    X(MODEL_STATIC, F_HAGAN, false) X(MODEL_STATIC, F_HAGAN, true) \
    X(MODEL_STATIC, F_OBLOJ, false) X(MODEL_STATIC, F_OBLOJ, true) \
    X(MODEL_STATIC, F_EXPANSION, false) X(MODEL_STATIC, F_EXPANSION, true) \
    X(MODEL_DYN_I, F_HAGAN, false) X(MODEL_DYN_I, F_HAGAN, true)   \
    X(MODEL_DYN_II, F_HAGAN, false) X(MODEL_DYN_II, F_HAGAN, true)

static int variant_index(int model, int formula, bool bfree) {
    int v = 0;
#define SABR_IDX(MD, FM, BF) \
    if (model == MD && (MD != MODEL_STATIC || formula == FM) && bfree == BF) return v; \
    ++v;
    SABR_FORMULA_VARIANTS(SABR_IDX)
#undef SABR_IDX
    return -1;
}

const void *objective_kernel_ptr(int model, int formula, bool fp32, bool bfree) {
    static const void *tab32[] = {
#define SABR_P(MD, FM, BF) (const void *)objective_kernel<MD, FM, float, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    static const void *tab64[] = {
#define SABR_P(MD, FM, BF) (const void *)objective_kernel<MD, FM, double, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    const int v = variant_index(model, formula, bfree);
    return v < 0 ? nullptr : (fp32 ? tab32[v] : tab64[v]);
}

const void *sa_kernel_ptr(int model, int formula, bool fp32, bool bfree, int lpc) {
    static const void *tab32[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, float, BF, 1>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    static const void *tab64[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, double, BF, 1>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    static const void *tab32x2[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, float, BF, 2>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    static const void *tab64x2[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, double, BF, 2>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    // wide lane groups: float dynamic models only (few chains, many rows)
#define SABR_WIDE(MD, BF)                                                                          \
    {(const void *)sa_kernel<MD, F_HAGAN, float, BF, 4>, (const void *)sa_kernel<MD, F_HAGAN, float, BF, 8>, \
     (const void *)sa_kernel<MD, F_HAGAN, float, BF, 16>}
    static const void *wide[4][3] = {SABR_WIDE(MODEL_DYN_I, false), SABR_WIDE(MODEL_DYN_I, true),
                                     SABR_WIDE(MODEL_DYN_II, false), SABR_WIDE(MODEL_DYN_II, true)};
#undef SABR_WIDE
    const int v = variant_index(model, formula, bfree);
    if (v < 0) return nullptr;
    if (lpc == 2) return fp32 ? tab32x2[v] : tab64x2[v];
    if (lpc == 4 || lpc == 8 || lpc == 16) {
        if (!fp32 || model == MODEL_STATIC) return nullptr;
        const int w = (model == MODEL_DYN_II ? 2 : 0) + (bfree ? 1 : 0);
        return wide[w][lpc == 4 ? 0 : (lpc == 8 ? 1 : 2)];
    }
    return lpc == 1 ? (fp32 ? tab32[v] : tab64[v]) : nullptr;
}

bool wide_lanes_supported(int model, bool fp32) { return fp32 && model != MODEL_STATIC; }

const void *polish_kernel_ptr(int model, int formula, bool bfree) {
    static const void *tab[] = {
#define SABR_P(MD, FM, BF) (const void *)polish_kernel<MD, FM, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    const int v = variant_index(model, formula, bfree);
    return v < 0 ? nullptr : tab[v];
}

// ---------------------------------------------------------------------------
// Start point from the at-the-money vols (Section 3, after eq. "sigma-SABR"):
// at K = f the static formulas give ln sigma_ATM = ln alpha - (1 - beta) ln f
// (up to the T-correction), so beta is one plus the slope of the least-squares
// line of ln sigma_ATM against ln f over the maturities, and alpha =
// f^(1 - beta) sigma_ATM.  sigma_ATM of a row is its market vol at K = f, linear
// in ln K between the two strikes around f (the end strike's vol beyond the
// row); beta is fitted only when it is calibrated and the forwards differ
// (else the fixed beta, or the centre of its box); alpha is taken at the
// shortest maturity (lowest index on ties), where the neglected T-correction
// is smallest; both are clamped to the box and every other coordinate is the
// box centre.  One wave: lane i % 64 takes maturity i, sums meet in a
// butterfly.
// ---------------------------------------------------------------------------
__device__ double atm_vol_of_row(int m, const double *K, const double *v, double f) {
#pragma clang fp contract(off)
    if (f <= K[0]) return v[0];
    if (f >= K[m - 1]) return v[m - 1];
    int j = 0;
    while (K[j + 1] < f) ++j;   // strikes of a row increase
    const double u = (log(f) - log(K[j])) / (log(K[j + 1]) - log(K[j]));
    return v[j] + u * (v[j + 1] - v[j]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(64) atm_seed_kernel(AtmDesc d, const double *T, const double *fwd,
                                                      const int32_t *offs, const double *K, const double *vol,
                                                      double *x0) {
#pragma clang fp contract(off)
    const int lane = threadIdx.x;
    double sx = 0.0, sy = 0.0, tmin = __builtin_inf();
    int imin = 0x7fffffff;
    bool distinct = false;
    for (int i = lane; i < d.n_mat; i += 64) {
        const double sa = atm_vol_of_row(offs[i + 1] - offs[i], K + offs[i], vol + offs[i], fwd[i]);
        sx += log(fwd[i]);
        sy += log(sa);
        if (T[i] < tmin) {
            tmin = T[i];
            imin = i;
        }
        distinct |= fwd[i] != fwd[0];
    }
    // shortest maturity, lowest index on ties
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double t2 = __shfl_xor(tmin, o, 64);
        const int i2 = __shfl_xor(imin, o, 64);
        if (t2 < tmin || (t2 == tmin && i2 < imin)) {
            tmin = t2;
            imin = i2;
        }
    }
    const double n = (double)d.n_mat;
    const double mx = wave_sum(sx) / n, my = wave_sum(sy) / n;
    double sxx = 0.0, sxy = 0.0;
    for (int i = lane; i < d.n_mat; i += 64) {
        const double sa = atm_vol_of_row(offs[i + 1] - offs[i], K + offs[i], vol + offs[i], fwd[i]);
        const double dx = log(fwd[i]) - mx;
        sxx += dx * dx;
        sxy += dx * (log(sa) - my);
    }
    sxx = wave_sum(sxx);
    sxy = wave_sum(sxy);
    const bool any_distinct = __ballot(distinct) != 0;
    if (lane != 0) return;
    const int np = d.n_par;
    double b = d.beta;
    if (d.beta_free) {
        b = 0.5 * (d.lb[np - 1] + d.ub[np - 1]);
        if (any_distinct && d.n_mat >= 2 && sxx > 0.0) b = fmin(fmax(1.0 + sxy / sxx, d.lb[np - 1]), d.ub[np - 1]);
    }
    const int s = imin;
    const double sa = atm_vol_of_row(offs[s + 1] - offs[s], K + offs[s], vol + offs[s], fwd[s]);
    const double a = pow(fwd[s], 1.0 - b) * sa;
    for (int k = 0; k < np; ++k) x0[k] = 0.5 * (d.lb[k] + d.ub[k]);
    x0[0] = fmin(fmax(a, d.lb[0]), d.ub[0]);
    if (d.beta_free) x0[np - 1] = b;
}

const void *atm_seed_kernel_ptr() { return (const void *)atm_seed_kernel; }
const void *prepare_points_kernel_ptr() { return (const void *)prepare_points_kernel; }
const void *prepare_mats_kernel_ptr() { return (const void *)prepare_mats_kernel; }

// (room for one spare record per row, which the wide annealing kernels use)
size_t grid_smem_bytes(bool fp32, int n_pts, int n_mat) {
    return fp32 ? pts_bytes<float>(n_pts + n_mat) + sizeof(Row<float>) * n_mat
                : pts_bytes<double>(n_pts + n_mat) + sizeof(Row<double>) * n_mat;
}
size_t sa_smem_fixed_bytes() { return sizeof(ArgminSmem) + 2 * kMaxPar * sizeof(double); }

}  // namespace sabr
