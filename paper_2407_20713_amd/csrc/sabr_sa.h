// sabr_sa.h -- device pieces of the synchronous annealing (Section 5) shared
// by the batch kernel and the serving kernels: proposal and Metropolis test
// in double without contraction, the level-end argmin with its
// cross-workgroup exchange, and the Levenberg-Marquardt polish.
#pragma once
#include "sabr_formula.h"

namespace sabr {

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

// The same decision from the raw random word w (u = (w + 1/2) 2^-32), taken
// in float wherever the float value of exp(-delta / T) is clearly on one side
// of u, else by the double test above.  Float error: -delta / T to 3 float
// roundings, the exponent at most 25 in size, so exp is within 8e-6 relative;
// the screen's margin is 3e-5, so the result always equals the double test.
// exp(-25) lies below the smallest uniform 2^-33: larger drops (and +inf or
// NaN objectives) are rejected outright.
__device__ __forceinline__ bool metropolis_w(double fy, double fx, uint32_t w, double Tk, float invTf) {
#pragma clang fp contract(off)
    const double delta = fy - fx;
    if (delta <= 0.0) return true;
    const float a = (float)(-delta) * invTf;
    if (!(a >= -25.0f)) return false;
    const float e = __builtin_amdgcn_exp2f(a * 1.44269504088896341f);
    const float uf = fmaf((float)w, 0x1p-32f, 0x1p-33f);
    if (uf < e * (1.0f - 3e-5f)) return true;
    if (uf > e * (1.0f + 3e-5f)) return false;
    return unit_u32(w) < exp(-delta / Tk);
}

// Float proposal (float annealing mode): the same reflection and clamp as
// propose_coord, on the float values the float objective sees.  The step is
// t hw with hw = h (ub - lb) and t = 2u - 1 = (2 (w >> 8) + 1) 2^-24 - 1 for
// the 24-bit uniform u = ((w >> 8) + 1/2) 2^-24: t is exact in float (an odd
// multiple of 2^-24 below 1 in size), so one fma gives it.  Each reflection is
// a min (max) with the reflected value, which lies on the far side of y
// exactly when y is outside the bound, so the result is the same as the
// branches of propose_coord; the clamp is a median of three.
__device__ __forceinline__ float propose_coord_f(float x, uint32_t w, float hw, float lb, float ub) {
    const float t = fmaf((float)(w >> 8), 0x1p-23f, 0x1p-24f - 1.0f);
    float y = fmaf(t, hw, x);
    y = fminf(y, ub - (y - ub));
    y = fmaxf(y, lb + (lb - y));
    return __builtin_amdgcn_fmed3f(y, lb, ub);
}

// Sum of a double over the LPC consecutive lanes of a lane group (LPC <= 16),
// with DPP lane moves: swaps inside quads (lane ^ 1, lane ^ 2), then the
// mirror inside each 8 and each 16 lanes.  Each step adds a value and its
// partner's in opposite orders on the two lanes of a pair, so every lane of
// the group ends with the same bits.
template <int DPP>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), DPP, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), DPP, 0xf, 0xf, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
template <int LPC>
__device__ __forceinline__ double group_sum(double v) {
    if constexpr (LPC >= 2) v = v + dpp_move<0xB1>(v);    // quad_perm [1,0,3,2]
    if constexpr (LPC >= 4) v = v + dpp_move<0x4E>(v);    // quad_perm [2,3,0,1]
    if constexpr (LPC >= 8) v = v + dpp_move<0x141>(v);   // row_half_mirror
    if constexpr (LPC >= 16) v = v + dpp_move<0x140>(v);  // row_mirror
    static_assert(LPC <= 16, "lane groups of at most 16 lanes");
    return v;
}

// Iterations [t_begin, t_end) of one chain at one temperature level (Section
// 5): proposal, objective, Metropolis test, best-so-far.  The LPC lanes of a
// chain draw the Philox blocks of LPC consecutive iterations at once (lane
// `sub` the blocks of iteration t0 + sub) and hand them round by shuffles,
// so a lane group draws each block once.  Double mode proposes in double from
// 32-bit uniforms; float mode proposes in float from 24-bit uniforms.
template <int NP, int NB, int LPC, typename R, typename FOBJ>
__device__ __forceinline__ void sa_level(int chain, int sub, int t_begin, int t_end, uint32_t k0, uint32_t k1,
                                         double h, double Tk, const double *s_lb, const double *s_ub, double *x,
                                         double &fx, double *bx, double &fb, unsigned long long &nacc, FOBJ f_of) {
    const float invTf = (float)(1.0 / Tk);
    // float mode keeps the chain's state in float through the level (every
    // state it can reach is a float proposal, or the start point, which the
    // float objective sees rounded anyway); x is updated at the end
    float xf[NP], lbf[NP], ubf[NP], hw[NP];
    bool moved = false;
    if constexpr (sizeof(R) == 4) {
#pragma unroll
        for (int c = 0; c < NP; ++c) {
            xf[c] = (float)x[c];
            lbf[c] = (float)s_lb[c];
            ubf[c] = (float)s_ub[c];
            hw[c] = (float)h * (ubf[c] - lbf[c]);
        }
    }
    for (int t0 = t_begin; t0 < t_end; t0 += LPC) {
        uint4 wm[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b)
            wm[b] = philox4x32_10(make_uint4((uint32_t)chain, (uint32_t)(t0 + sub), (uint32_t)b, 1u), k0, k1);
        const int kn = min(LPC, t_end - t0);
        // the NP + 1 words of iteration t0 + k come from lane k of the group;
        // the next iteration's are fetched before this one's objective
        constexpr int NW = NP + 1;
        auto fetch = [&](int k, uint32_t *w) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                const uint4 &v = wm[i / 4];
                const uint32_t word = (i % 4 == 0) ? v.x : (i % 4 == 1) ? v.y : (i % 4 == 2) ? v.z : v.w;
                if constexpr (LPC > 1)
                    w[i] = __shfl(word, k, LPC);
                else
                    w[i] = word;
            }
        };
        uint32_t w[NW], wn[NW];
        fetch(0, w);
#pragma unroll 1
        for (int k = 0; k < kn; ++k) {
            if (k + 1 < kn) fetch(k + 1, wn);
            if constexpr (sizeof(R) == 4) {
                float y[NP];
#pragma unroll
                for (int c = 0; c < NP; ++c) y[c] = propose_coord_f(xf[c], w[c], hw[c], lbf[c], ubf[c]);
                const double fy = f_of(y);
                if (metropolis_w(fy, fx, w[NP], Tk, invTf)) {
#pragma unroll
                    for (int c = 0; c < NP; ++c) xf[c] = y[c];
                    moved = true;
                    fx = fy;
                    ++nacc;
                    if (fy < fb) {
                        fb = fy;
#pragma unroll
                        for (int c = 0; c < NP; ++c) bx[c] = (double)y[c];
                    }
                }
            } else {
                double y[NP];
#pragma unroll
                for (int c = 0; c < NP; ++c) y[c] = propose_coord(x[c], unit_u32(w[c]), h, s_lb[c], s_ub[c]);
                const double fy = f_of(y);
                if (metropolis_w(fy, fx, w[NP], Tk, invTf)) {
#pragma unroll
                    for (int c = 0; c < NP; ++c) x[c] = y[c];
                    fx = fy;
                    ++nacc;
                    if (fy < fb) {
                        fb = fy;
#pragma unroll
                        for (int c = 0; c < NP; ++c) bx[c] = y[c];
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) w[i] = wn[i];
        }
    }
    if constexpr (sizeof(R) == 4) {
        if (moved) {
#pragma unroll
            for (int c = 0; c < NP; ++c) x[c] = (double)xf[c];
        }
    }
}

// Wave-level argmin of (f, id): smaller f, ties to the smaller id (a total
// order, so any pairing of the lanes gives the same winner).  Inside each 16
// lanes by DPP moves (quad swaps, half-row and row mirrors), across the rows
// by two lane shuffles.  Every lane of the wave takes part.
template <int DPP>
__device__ __forceinline__ int dpp_move_i(int v) { return __builtin_amdgcn_mov_dpp(v, DPP, 0xf, 0xf, false); }
__device__ __forceinline__ void argmin_step(double &f, int &id, double fo, int io) {
    if (fo < f || (fo == f && io < id)) {
        f = fo;
        id = io;
    }
}
__device__ __forceinline__ void wave_argmin(double &f, int &id) {
    argmin_step(f, id, dpp_move<0xB1>(f), dpp_move_i<0xB1>(id));
    argmin_step(f, id, dpp_move<0x4E>(f), dpp_move_i<0x4E>(id));
    argmin_step(f, id, dpp_move<0x141>(f), dpp_move_i<0x141>(id));
    argmin_step(f, id, dpp_move<0x140>(f), dpp_move_i<0x140>(id));
    argmin_step(f, id, __shfl_xor(f, 16, 64), __shfl_xor(id, 16, 64));
    argmin_step(f, id, __shfl_xor(f, 32, 64), __shfl_xor(id, 32, 64));
}

struct ArgminSmem {
    double wf[16];
    int wid[16];
    double bf;
    int bid;
    int fail;   // a wait of the exchange timed out
    double bx[kMaxPar];
    double wx[kWG / 64][kMaxPar];   // each wave's winner (exchange read by a whole workgroup)
    uint32_t rp[kMaxReaders][3 + 2 * kMaxPar];   // the reader workgroups' results
};

// Level-end argmin over every chain of the request (workgroups of one request
// exchange candidates through device memory).  Afterwards every thread sees
// the winner in s.bf / s.bx.  `round` counts exchanges; slots alternate
// between two halves so that a fast workgroup can never overwrite a slot
// another one has not read yet (it publishes round r + 2 only after every
// workgroup has published round r + 1, which each does after reading round
// r).  The first wave of each workgroup publishes its candidate as tagged
// words (lane k stores word k).  Up to 64 workgroups, the first wave of each
// then watches the request's slots (lane w slot w), reading every word of a
// slot at once until all show the round.  Beyond 64, each of the request's
// first R = ceil(workgroups / 256) workgroups reads 256 slots (one per
// thread), takes their argmin and publishes it in its result slot (R of
// them for each round parity); every workgroup then reads the R results
// (thread r result r) and takes their argmin: the same result with traffic
// linear, not quadratic, in the workgroups, two trips after the last
// candidate is published.  Returns false, with *err set,
// if a slot did not show the round within the wait bound (the caller then
// ends).
template <int NP>
__device__ inline bool request_argmin(double f, int chain, bool active, const double *x, ArgminSmem &s,
                                      const ReqDesc &rq, int wg_local, int round, Cand *cands, int32_t *err) {
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
        s.fail = 0;
    }
    __syncthreads();
    if (active && chain == s.bid) {
#pragma unroll
        for (int k = 0; k < NP; ++k) s.bx[k] = x[k];
    }
    __syncthreads();
    if (rq.n_wg > 1) {
        constexpr int NW = 3 + 2 * NP;   // words of a candidate
        Cand *half = cands + rq.cand_off + (round & 1) * rq.n_wg;
        const uint32_t tag32 = (uint32_t)(round + 1);
        const uint64_t tag = (uint64_t)tag32 << 32;
        // words: f (low, high), chain, then x[i] (low, high)
        auto word_of = [&](int k) -> uint32_t {
            if (k == 2) return (uint32_t)s.bid;
            const uint64_t b = __builtin_bit_cast(uint64_t, k < 2 ? s.bf : s.bx[k < 3 ? 0 : (k - 3) >> 1]);
            const bool high = k < 2 ? k == 1 : ((k - 3) & 1) == 1;
            return high ? (uint32_t)(b >> 32) : (uint32_t)b;
        };
        // reads every word of a slot in one trip until all show the round
        // (false if the wait bound ran out)
        auto poll = [&](const Cand *slot, uint32_t *pay) -> bool {
            for (int spins = 0; spins < rq.spin_limit; ++spins) {
                uint64_t v[NW];
#pragma unroll
                for (int k = 0; k < NW; ++k)
                    v[k] = __hip_atomic_load(&slot->w[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_sched_barrier(0);
                bool all = true;
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    pay[k] = (uint32_t)v[k];
                    all &= (uint32_t)(v[k] >> 32) == tag32;
                }
                if (all) return true;
                __builtin_amdgcn_s_sleep(1);
            }
            return false;
        };
        auto pay_f = [](const uint32_t *pay) { return __builtin_bit_cast(double, ((uint64_t)pay[1] << 32) | pay[0]); };
        auto pay_x = [](const uint32_t *pay, int k) {
            return __builtin_bit_cast(double, ((uint64_t)pay[4 + 2 * k] << 32) | pay[3 + 2 * k]);
        };
        if (threadIdx.x < NW)
            __hip_atomic_store(&half[wg_local].w[threadIdx.x], tag | word_of(threadIdx.x), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        // the lanes that read candidate slots: for up to 64 workgroups the
        // first wave of every workgroup (lane w slot w); beyond that the
        // threads of the first R workgroups (thread t of workgroup r slot
        // 256 r + t), each of which publishes its argmin in a result slot
        const bool direct = rq.n_wg <= 64;
        const int nr = direct ? 0 : (rq.n_wg + (int)blockDim.x - 1) / (int)blockDim.x;
        Cand *res = cands + rq.cand_off + 2 * rq.n_wg + (round & 1) * nr;
        const bool reader = direct ? threadIdx.x < 64 : wg_local < nr;
        if (reader) {
            double cf = __builtin_inf();
            int cid = 0x7fffffff;
            double cx[NP];
#pragma unroll
            for (int k = 0; k < NP; ++k) cx[k] = 0.0;
            const int w = (direct ? 0 : wg_local * (int)blockDim.x) + (int)threadIdx.x;
            if (w < rq.n_wg) {
                uint32_t pay[NW];
                if (poll(&half[w], pay)) {
                    cf = pay_f(pay);
                    cid = (int)pay[2];
#pragma unroll
                    for (int k = 0; k < NP; ++k) cx[k] = pay_x(pay, k);
                } else {
                    __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s.fail = 1;
                }
            }
            int key = cid;
            double kf = cf;
            wave_argmin(kf, key);
            const unsigned long long m = __ballot(cid == key && cf == kf);
            const int src = __ffsll((long long)m) - 1;
            if (direct) {
                if (threadIdx.x == src) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) s.bx[k] = cx[k];
                    s.bf = kf;
                    s.bid = key;
                }
            } else {
                // every wave's winner, then the workgroup's, then its result slot
                const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
                if (lane == src) {
                    s.wf[wave] = kf;
                    s.wid[wave] = key;
#pragma unroll
                    for (int k = 0; k < NP; ++k) s.wx[wave][k] = cx[k];
                }
                __syncthreads();
                if (threadIdx.x == 0) {
                    int bw = 0;
                    for (int v = 1; v < (int)(blockDim.x >> 6); ++v)
                        if (s.wf[v] < s.wf[bw] || (s.wf[v] == s.wf[bw] && s.wid[v] < s.wid[bw])) bw = v;
                    s.bf = s.wf[bw];
                    s.bid = s.wid[bw];
                    for (int k = 0; k < NP; ++k) s.bx[k] = s.wx[bw][k];
                }
                __syncthreads();
                if (threadIdx.x < NW)
                    __hip_atomic_store(&res[wg_local].w[threadIdx.x], tag | word_of(threadIdx.x), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        if (!direct) {
            // the R results, one per thread, then their argmin
            if ((int)threadIdx.x < nr && !poll(&res[threadIdx.x], s.rp[threadIdx.x])) {
                __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s.fail = 1;
            }
            __syncthreads();
            if (threadIdx.x == 0 && s.fail == 0) {
                int br = 0;
                for (int r = 1; r < nr; ++r) {
                    const double fr = pay_f(s.rp[r]), fb = pay_f(s.rp[br]);
                    if (fr < fb || (fr == fb && (int)s.rp[r][2] < (int)s.rp[br][2])) br = r;
                }
                s.bf = pay_f(s.rp[br]);
                s.bid = (int)s.rp[br][2];
                for (int k = 0; k < NP; ++k) s.bx[k] = pay_x(s.rp[br], k);
            }
        }
        __syncthreads();
    }
    return s.fail == 0;
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
__device__ inline double lm_f(const double *v, const Pt<double> *pts, const Row<double> *rows, const int32_t *prow,
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

// One wave (threads 0..63 of the block) polishes x in place; returns f(x) and
// counts objective evaluations in *ne.
template <int MODEL, int FORMULA, bool BFREE>
__device__ inline double lm_polish(double *xio, const Pt<double> *pts, const Row<double> *rows, const int32_t *prow,
                            const ReqDesc &rq, unsigned long long *ne_out) {
    constexpr int NP = base_npar<MODEL>() + (BFREE ? 1 : 0);
    const int n = rq.n_pts;
    double x[NP], lb[NP], ub[NP], h[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        x[k] = xio[k];
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
#pragma unroll
    for (int k = 0; k < NP; ++k) xio[k] = x[k];
    *ne_out = ne;
    return fx;
}

}  // namespace sabr
