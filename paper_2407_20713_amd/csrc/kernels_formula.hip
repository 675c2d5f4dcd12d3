// kernels_formula.hip -- grid normalisation, batch objective, persistent
// synchronous annealing and compass polish (Sections 2, 3 and 5).
#include "sabr_formula.h"
#include "sabr_kernels.h"

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
    const double k = K[j], f = fwd_of_pt[j], beta = beta_of_pt[j];
    const double omb = 1.0 - beta;
    const double l = log(f / k);
    const double lk = log(k * f);
    const double kf = exp(0.5 * omb * lk);
    const double l2 = l * l;
    const double den = 1.0 + omb * omb / 24.0 * l2 + omb * omb * omb * omb / 1920.0 * l2 * l2;
    lfk[j] = l;
    lkf[j] = lk;
    Q1[j] = 1.0 / kf;
    Q2[j] = 1.0 / (kf * kf);
    if (formula_of_pt[j] == F_OBLOJ) {
        // z = (nu/alpha) f^(1-b) l / g(u), leading factor alpha g(u) / f^(1-b),
        // g(u) = u / (1 - e^-u), u = (1-b) l.
        const double F1 = exp(omb * log(f));
        const double u = omb * l;
        const double g = (u == 0.0) ? 1.0 : u / (-expm1(-u));
        P1[j] = g / (F1 * den);
        Z[j] = F1 * l / g;
    } else {
        P1[j] = 1.0 / (kf * den);
        Z[j] = kf * l;
    }
    const double t = target ? target[j] : 0.0;
    sw[j] = (weighting_of_pt[j] == W_RELATIVE) ? 1.0 / t : 1.0;
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
    Row<R> *rows = reinterpret_cast<Row<R> *>(smem + sizeof(Pt<R>) * rq.n_pts);
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
// Annealing arithmetic in double, evaluated exactly as written (no
// contraction), so that float-free runs take the same decisions as any other
// exact implementation of the same reading.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double propose_coord(double x, double u, double h, double lb, double ub) {
#pragma clang fp contract(off)
    double y = x + (h * (2.0 * u - 1.0)) * (ub - lb);
    if (y > ub) y = ub - (y - ub);
    if (y < lb) y = lb + (lb - y);
    if (y > ub) y = ub;
    if (y < lb) y = lb;
    return y;
}

__device__ __forceinline__ bool metropolis(double fy, double fx, double u, double Tk) {
#pragma clang fp contract(off)
    const double delta = fy - fx;
    return delta <= 0.0 || u < exp(-delta / Tk);
}

// Wave-level argmin of (f, id): smaller f, ties to the smaller id.
__device__ __forceinline__ void wave_argmin(double &f, int &id) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double fo = __shfl_xor(f, off, 64);
        const int io = __shfl_xor(id, off, 64);
        if (fo < f || (fo == f && io < id)) {
            f = fo;
            id = io;
        }
    }
}

struct ArgminSmem {
    double wf[kWG / 64];
    int wid[kWG / 64];
    double bf;
    int bid;
    int pad;
    double bx[kMaxPar];
};

// Level-end argmin over every chain of the request (workgroups of one request
// exchange candidates through device memory and a counter).  Afterwards every
// thread sees the winner in s.bf / s.bx.  `round` counts exchanges; slots
// alternate between two halves so that a fast workgroup can never overwrite
// a slot another one has not read yet.
template <int NP>
__device__ void request_argmin(double f, int chain, bool active, const double *x, ArgminSmem &s,
                               const ReqDesc &rq, int wg_local, int round, Cand *cands, uint32_t *bar,
                               int req, int32_t *err) {
    double wf = active ? f : __builtin_inf();
    int wid = active ? chain : 0x7fffffff;
    wave_argmin(wf, wid);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        s.wf[wave] = wf;
        s.wid[wave] = wid;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double bf = s.wf[0];
        int bid = s.wid[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
            if (s.wf[w] < bf || (s.wf[w] == bf && s.wid[w] < bid)) {
                bf = s.wf[w];
                bid = s.wid[w];
            }
        s.bf = bf;
        s.bid = bid;
    }
    __syncthreads();
    if (active && chain == s.bid) {
#pragma unroll
        for (int k = 0; k < NP; ++k) s.bx[k] = x[k];
    }
    __syncthreads();
    if (rq.n_wg > 1) {
        if (threadIdx.x == 0) {
            Cand *half = cands + rq.cand_off + (round & 1) * rq.n_wg;
            Cand &c = half[wg_local];
            c.f = s.bf;
            c.chain = s.bid;
            for (int k = 0; k < NP; ++k) c.x[k] = s.bx[k];
            __hip_atomic_fetch_add(&bar[req], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t want = (uint32_t)(round + 1) * (uint32_t)rq.n_wg;
            int spins = 0;
            while (__hip_atomic_load(&bar[req], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < want) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > (1 << 24)) {
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            int best = 0;
            double bf = __hip_atomic_load(&half[0].f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int bid = __hip_atomic_load(&half[0].chain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int w = 1; w < rq.n_wg; ++w) {
                const double fw = __hip_atomic_load(&half[w].f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int iw = __hip_atomic_load(&half[w].chain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (fw < bf || (fw == bf && iw < bid)) {
                    bf = fw;
                    bid = iw;
                    best = w;
                }
            }
            s.bf = bf;
            s.bid = bid;
            for (int k = 0; k < NP; ++k)
                s.bx[k] = __hip_atomic_load(&half[best].x[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Persistent synchronous annealing (Section 5, Technique I).  One lane is
// one Markov chain; the workgroups of a request exchange their best state
// at each level end; every chain restarts from the request's best.
// ---------------------------------------------------------------------------
template <int MODEL, int FORMULA, typename R, bool BFREE>
__global__ void __launch_bounds__(kWG) sa_kernel(const ReqDesc *reqs, const int32_t *wg_req,
                                                 PointsD P, MatsD Mt, const double *sched_g,
                                                 const double *sched_h, Cand *cands, uint32_t *bar,
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
    Row<R> *rows = reinterpret_cast<Row<R> *>(reinterpret_cast<unsigned char *>(pts) + sizeof(Pt<R>) * rq.n_pts);
    stage_grid<R>(rq, P, Mt, pts, rows);
    if (threadIdx.x < NP) {
        s_lb[threadIdx.x] = rq.lb[threadIdx.x];
        s_ub[threadIdx.x] = rq.ub[threadIdx.x];
    }
    __syncthreads();

    const int wg_local = blockIdx.x - rq.wg_first;
    const int chain = wg_local * kWG + threadIdx.x;
    const bool active = chain < rq.n_chains;
    const int n_mat = rq.n_mat, L = rq.chain_len, n_iters = rq.n_iters;
    const double beta = rq.beta, tmax = rq.t_max;
    const uint32_t k0 = rq.key0, k1 = rq.key1;

    double x[NP], bx[NP], y[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) x[k] = bx[k] = rq.x0[k];
    double fx = objective<MODEL, FORMULA, R, BFREE, false>(x, pts, rows, n_mat, beta, tmax, nullptr);
    const double T0 = rq.T0 > 0.0 ? rq.T0 : ((fx > 0.0 && fx < __builtin_inf()) ? fx : 1.0);
    double fb = fx;
    unsigned long long nacc = 0;
    int round = 0;

    for (int lev = 0; lev < rq.n_levels; ++lev) {
        const double g = sched_g[rq.sched_off + lev];
        const double h = sched_h[rq.sched_off + lev];
        const double Tk = T0 * g;
        const int t1 = min((lev + 1) * L, n_iters);
        if (active) {
            for (int t = lev * L; t < t1; ++t) {
                double u[NB * 4];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const uint4 w = philox4x32_10(make_uint4((uint32_t)chain, (uint32_t)t, (uint32_t)b, 1u), k0, k1);
                    u[4 * b + 0] = unit_u32(w.x);
                    u[4 * b + 1] = unit_u32(w.y);
                    u[4 * b + 2] = unit_u32(w.z);
                    u[4 * b + 3] = unit_u32(w.w);
                }
#pragma unroll
                for (int k = 0; k < NP; ++k) y[k] = propose_coord(x[k], u[k], h, s_lb[k], s_ub[k]);
                const double fy = objective<MODEL, FORMULA, R, BFREE, false>(y, pts, rows, n_mat, beta, tmax, nullptr);
                if (metropolis(fy, fx, u[NP], Tk)) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) x[k] = y[k];
                    fx = fy;
                    ++nacc;
                    if (fy < fb) {
                        fb = fy;
#pragma unroll
                        for (int k = 0; k < NP; ++k) bx[k] = y[k];
                    }
                }
            }
        }
        request_argmin<NP>(fx, chain, active, x, am, rq, wg_local, round++, cands, bar, req, err);
        fx = am.bf;
#pragma unroll
        for (int k = 0; k < NP; ++k) x[k] = am.bx[k];
        __syncthreads();
    }
    // best-so-far over all chains of the request
    request_argmin<NP>(fb, chain, active, bx, am, rq, wg_local, round++, cands, bar, req, err);
    // accepted moves: workgroup sum, one integer atomic per workgroup
    unsigned long long a = active ? nacc : 0ull;
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

// ---------------------------------------------------------------------------
// Compass-search polish in double from the annealing result: lane l < 2 NP
// evaluates x +/- s_j e_j (j = l/2, + for even l), the lowest improving lane
// wins, no improvement halves every step.  One wave per request.
// ---------------------------------------------------------------------------
template <int MODEL, int FORMULA, bool BFREE>
__global__ void __launch_bounds__(64) polish_kernel(const ReqDesc *reqs, const int32_t *req_ids,
                                                    PointsD P, MatsD Mt, ChainOut *best,
                                                    unsigned long long *evals) {
    constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
    extern __shared__ unsigned char smem[];
    const int req = req_ids[blockIdx.x];
    const ReqDesc &rq = reqs[req];
    Pt<double> *pts = reinterpret_cast<Pt<double> *>(smem);
    Row<double> *rows = reinterpret_cast<Row<double> *>(smem + sizeof(Pt<double>) * rq.n_pts);
    stage_grid<double>(rq, P, Mt, pts, rows);
    __syncthreads();
    const int lane = threadIdx.x;
    double x[NP], s[NP], y[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        x[k] = best[req].bx[k];
        s[k] = 1e-2 * (rq.ub[k] - rq.lb[k]);
    }
    double fx = objective<MODEL, FORMULA, double, BFREE, false>(x, pts, rows, rq.n_mat, rq.beta, rq.t_max, nullptr);
    unsigned long long ne = 1;
    const int j = lane >> 1;
    for (int round = 0; round < 200; ++round) {
        if (s[0] < 1e-10 * (rq.ub[0] - rq.lb[0])) break;
        double fy = __builtin_inf();
#pragma unroll
        for (int k = 0; k < NP; ++k) y[k] = x[k];
        if (lane < 2 * NP) {
#pragma unroll
            for (int k = 0; k < NP; ++k)
                if (k == j) {
                    double v = (lane & 1) ? x[k] - s[k] : x[k] + s[k];
                    v = fmin(fmax(v, rq.lb[k]), rq.ub[k]);
                    y[k] = v;
                }
            fy = objective<MODEL, FORMULA, double, BFREE, false>(y, pts, rows, rq.n_mat, rq.beta, rq.t_max, nullptr);
        }
        ne += 2 * NP;
        const unsigned long long m = __ballot(lane < 2 * NP && fy < fx);
        if (m) {
            const int w = __ffsll((long long)m) - 1;
            fx = __shfl(fy, w, 64);
#pragma unroll
            for (int k = 0; k < NP; ++k) x[k] = __shfl(y[k], w, 64);
        } else {
#pragma unroll
            for (int k = 0; k < NP; ++k) s[k] *= 0.5;
        }
    }
    if (lane == 0) {
        best[req].bf = fx;
        for (int k = 0; k < NP; ++k) best[req].bx[k] = x[k];
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

const void *sa_kernel_ptr(int model, int formula, bool fp32, bool bfree) {
    static const void *tab32[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, float, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    static const void *tab64[] = {
#define SABR_P(MD, FM, BF) (const void *)sa_kernel<MD, FM, double, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    const int v = variant_index(model, formula, bfree);
    return v < 0 ? nullptr : (fp32 ? tab32[v] : tab64[v]);
}

const void *polish_kernel_ptr(int model, int formula, bool bfree) {
    static const void *tab[] = {
#define SABR_P(MD, FM, BF) (const void *)polish_kernel<MD, FM, BF>,
        SABR_FORMULA_VARIANTS(SABR_P)
#undef SABR_P
    };
    const int v = variant_index(model, formula, bfree);
    return v < 0 ? nullptr : tab[v];
}

const void *prepare_points_kernel_ptr() { return (const void *)prepare_points_kernel; }
const void *prepare_mats_kernel_ptr() { return (const void *)prepare_mats_kernel; }

size_t grid_smem_bytes(bool fp32, int n_pts, int n_mat) {
    return fp32 ? sizeof(Pt<float>) * n_pts + sizeof(Row<float>) * n_mat
                : sizeof(Pt<double>) * n_pts + sizeof(Row<double>) * n_mat;
}
size_t sa_smem_fixed_bytes() { return sizeof(ArgminSmem) + 2 * kMaxPar * sizeof(double); }

}  // namespace sabr
