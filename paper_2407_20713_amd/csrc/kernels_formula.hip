// kernels_formula.hip -- grid normalisation, batch objective, persistent
// synchronous annealing and Levenberg-Marquardt polish (Sections 2, 3 and 5).
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
        Cand *half = cands + rq.cand_off + (round & 1) * rq.n_wg;
        if (threadIdx.x == 0) {
            Cand &c = half[wg_local];
            c.f = s.bf;
            c.chain = s.bid;
            for (int k = 0; k < NP; ++k) c.x[k] = s.bx[k];
            __hip_atomic_fetch_add(&bar[req * kBarStride], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t want = (uint32_t)(round + 1) * (uint32_t)rq.n_wg;
            int spins = 0;
            while (__hip_atomic_load(&bar[req * kBarStride], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < want) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1 << 24)) {
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        // the first wave reads every candidate at once and takes their argmin
        if (threadIdx.x < 64) {
            double cf = __builtin_inf();
            int cid = 0x7fffffff, cw = 0;
            for (int w = threadIdx.x; w < rq.n_wg; w += 64) {
                const double fw = __hip_atomic_load(&half[w].f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const int iw = __hip_atomic_load(&half[w].chain, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (fw < cf || (fw == cf && iw < cid)) {
                    cf = fw;
                    cid = iw;
                    cw = w;
                }
            }
            int key = cid;
            double kf = cf;
            wave_argmin(kf, key);
            // the lane holding the winning chain id names its workgroup
            const unsigned long long m = __ballot(cid == key && cf == kf);
            const int src = __ffsll((long long)m) - 1;
            const int bw = __shfl(cw, src, 64);
            if (threadIdx.x < NP)
                s.bx[threadIdx.x] = __hip_atomic_load(&half[bw].x[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (threadIdx.x == 0) {
                s.bf = kf;
                s.bid = key;
            }
        }
        __syncthreads();
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

    // LPC lanes share one chain: each takes every LPC-th strike and the
    // partial sums are combined across the lane group; the chain state and
    // its random words are the same on every lane of the group.
    const int wg_local = blockIdx.x - rq.wg_first;
    const int sub = threadIdx.x % LPC;
    const int chain = wg_local * (kWG / LPC) + threadIdx.x / LPC;
    const bool active = chain < rq.n_chains;
    const int n_mat = rq.n_mat, L = rq.chain_len, n_iters = rq.n_iters;
    const double beta = rq.beta, tmax = rq.t_max;
    const uint32_t k0 = rq.key0, k1 = rq.key1;
    auto f_of = [&](const double *v) {
        double part = objective<MODEL, FORMULA, R, BFREE, false, LPC>(v, pts, rows, n_mat, beta, tmax, nullptr, sub);
        if constexpr (LPC == 2) part = part + __shfl_xor(part, 1, 64);
        return part;
    };

    double x[NP], bx[NP], y[NP];
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
                const double fy = f_of(y);
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

// ---------------------------------------------------------------------------
// Levenberg-Marquardt polish in double from the annealing result (one wave
// per request, lane = grid point).  Residuals r_j = (target - sigma_j) s_j;
// Jacobian by central differences with h_k = 6e-6 (ub_k - lb_k) clamped to
// the box; step (J^T J + lambda diag(J^T J)) d = -J^T r solved by Cholesky,
// y = clamp(x + d); accept if f(y) < f(x) (lambda /= 10, floor 1e-15), else
// lambda *= 10, up to 12 tries; at most 60 iterations; stop at f = 0, when no
// damping helps, or when a step gains less than 1e-15 f.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum_bcast(T v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return __shfl(v, 0, 64);   // one association order for every lane
}

// Sum of squared residuals at v over the lane's points; `ok` false if any
// model vol is not finite and positive (or v is an infeasible case II vector).
template <int MODEL, int FORMULA, bool BFREE>
__device__ double lm_f(const double *v, const Pt<double> *pts, const Row<double> *rows, const int32_t *prow,
                       int n_pts, const ReqDesc &rq, bool &ok) {
    ModelEval<MODEL, FORMULA, double, BFREE> ev;
    bool good = ev.init(v, rq.beta, rq.t_max);
    double acc = 0.0;
    for (int j = threadIdx.x; j < n_pts && good; j += 64) {
        ev.row(rows[prow[j]]);
        const double sig = ev.point(pts[j]);
        good &= vol_ok(sig);
        const double e = fma(-sig, pts[j].sw, pts[j].tsw);
        acc = fma(e, e, acc);
    }
    ok = __ballot(!good) == 0ull;
    return wave_sum_bcast(acc);
}

template <int NP>
__device__ __forceinline__ bool cholesky_solve(const double *A, const double *g, double lambda, double *d) {
    double Mx[NP * NP], L[NP * NP], yv[NP];
    double tr = 0.0;
#pragma unroll
    for (int k = 0; k < NP; ++k) tr += A[k * NP + k];
    const double fl = 1e-12 * tr / NP + 1e-300;
#pragma unroll
    for (int a = 0; a < NP * NP; ++a) Mx[a] = A[a];
#pragma unroll
    for (int k = 0; k < NP; ++k) Mx[k * NP + k] += lambda * fmax(A[k * NP + k], fl);
#pragma unroll
    for (int a = 0; a < NP; ++a)
#pragma unroll
        for (int b = 0; b <= a; ++b) {
            double s = Mx[a * NP + b];
#pragma unroll
            for (int k = 0; k < b; ++k) s -= L[a * NP + k] * L[b * NP + k];
            if (a == b) {
                if (!(s > 0.0)) return false;
                L[a * NP + a] = sqrt(s);
            } else {
                L[a * NP + b] = s / L[b * NP + b];
            }
        }
#pragma unroll
    for (int a = 0; a < NP; ++a) {
        double s = -g[a];
#pragma unroll
        for (int k = 0; k < a; ++k) s -= L[a * NP + k] * yv[k];
        yv[a] = s / L[a * NP + a];
    }
#pragma unroll
    for (int a = NP - 1; a >= 0; --a) {
        double s = yv[a];
#pragma unroll
        for (int k = a + 1; k < NP; ++k) s -= L[k * NP + a] * d[k];
        d[a] = s / L[a * NP + a];
    }
    return true;
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
    Row<double> *rows = reinterpret_cast<Row<double> *>(smem + sizeof(Pt<double>) * rq.n_pts);
    int32_t *prow = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(rows) + sizeof(Row<double>) * rq.n_mat);
    stage_grid<double>(rq, P, Mt, pts, rows);
    __syncthreads();
    for (int i = 0; i < rq.n_mat; ++i)
        for (int j = rows[i].p0 + threadIdx.x; j < rows[i].p1; j += 64) prow[j] = i;
    __syncthreads();
    const int n = rq.n_pts;
    double x[NP], lb[NP], ub[NP], h[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        x[k] = best[req].bx[k];
        lb[k] = rq.lb[k];
        ub[k] = rq.ub[k];
        h[k] = 6e-6 * (ub[k] - lb[k]);
    }
    bool ok;
    double fx = lm_f<MODEL, FORMULA, BFREE>(x, pts, rows, prow, n, rq, ok);
    unsigned long long ne = 1;
    if (!ok) fx = __builtin_inf();
    double lambda = 1e-3;
    for (int it = 0; it < 60 && fx > 0.0 && fx < __builtin_inf(); ++it) {
        double A[NP * NP], g[NP];
#pragma unroll
        for (int a = 0; a < NP * NP; ++a) A[a] = 0.0;
#pragma unroll
        for (int a = 0; a < NP; ++a) g[a] = 0.0;
        for (int j = threadIdx.x; j < n; j += 64) {
            const Row<double> rw = rows[prow[j]];
            const Pt<double> pj = pts[j];
            ModelEval<MODEL, FORMULA, double, BFREE> ev;
            ev.init(x, rq.beta, rq.t_max);
            ev.row(rw);
            const double r0 = fma(-ev.point(pj), pj.sw, pj.tsw);
            double Jr[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                double xp[NP], xm[NP];
#pragma unroll
                for (int m = 0; m < NP; ++m) xp[m] = xm[m] = x[m];
                xp[k] = fmin(fmax(x[k] + h[k], lb[k]), ub[k]);
                xm[k] = fmin(fmax(x[k] - h[k], lb[k]), ub[k]);
                const double den = xp[k] - xm[k];
                ModelEval<MODEL, FORMULA, double, BFREE> ep, em;
                const bool okp = ep.init(xp, rq.beta, rq.t_max), okm = em.init(xm, rq.beta, rq.t_max);
                ep.row(rw);
                em.row(rw);
                const double sp = ep.point(pj), sm = em.point(pj);
                const double rp = fma(-sp, pj.sw, pj.tsw), rm = fma(-sm, pj.sw, pj.tsw);
                const bool good = okp && okm && den > 0.0 && vol_ok(sp) && vol_ok(sm);
                Jr[k] = good ? (rp - rm) / den : 0.0;
            }
#pragma unroll
            for (int a = 0; a < NP; ++a) {
                g[a] = fma(Jr[a], r0, g[a]);
#pragma unroll
                for (int b = 0; b < NP; ++b) A[a * NP + b] = fma(Jr[a], Jr[b], A[a * NP + b]);
            }
        }
        ne += 2 * NP;
#pragma unroll
        for (int a = 0; a < NP * NP; ++a) A[a] = wave_sum_bcast(A[a]);
#pragma unroll
        for (int a = 0; a < NP; ++a) g[a] = wave_sum_bcast(g[a]);
        bool moved = false;
        double fnew = fx;
        for (int tries = 0; tries < 12; ++tries) {
            double d[NP], y[NP];
            if (cholesky_solve<NP>(A, g, lambda, d)) {
#pragma unroll
                for (int k = 0; k < NP; ++k) y[k] = fmin(fmax(x[k] + d[k], lb[k]), ub[k]);
                bool oky;
                const double fy = lm_f<MODEL, FORMULA, BFREE>(y, pts, rows, prow, n, rq, oky);
                ++ne;
                if (oky && fy < fx) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) x[k] = y[k];
                    fnew = fy;
                    lambda = fmax(lambda / 10.0, 1e-15);
                    moved = true;
                    break;
                }
            }
            lambda *= 10.0;
        }
        if (!moved) break;
        const double gain = fx - fnew;
        fx = fnew;
        if (gain <= 1e-15 * fx) break;
    }
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
    const int v = variant_index(model, formula, bfree);
    if (v < 0) return nullptr;
    if (lpc == 2) return fp32 ? tab32x2[v] : tab64x2[v];
    return fp32 ? tab32[v] : tab64[v];
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
