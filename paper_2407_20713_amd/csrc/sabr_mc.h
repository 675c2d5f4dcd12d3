// sabr_mc.h -- device pieces of the Monte Carlo path (Section 4, eq.
// "dis_SABRd") shared by the batch kernels and the serving kernels.
#pragma once
#include "sabr_dev.h"
#include "sabr_kernels.h"

namespace sabr {

constexpr double kLog2Abs = -99.657842846620870436109582884681;   // log2(1e-30)

template <typename R> struct MC;
template <> struct MC<float> {
    static __device__ __forceinline__ float exp2_(float v) { return __builtin_amdgcn_exp2f(v); }
    // Box-Muller: r = sqrt(-2 ln u1), (cos 2 pi u2, sin 2 pi u2); the hardware
    // sine and cosine take their argument in revolutions.
    static __device__ __forceinline__ void normals(float u1, float u2, float &z1, float &z2) {
        const float r = __builtin_amdgcn_sqrtf(-2.0f * kLn2f * __builtin_amdgcn_logf(u1));
        z1 = r * __builtin_amdgcn_cosf(u2);
        z2 = r * __builtin_amdgcn_sinf(u2);
    }
    static __device__ __forceinline__ float unit(uint32_t w) { return unit_u24f(w); }
};
template <> struct MC<double> {
    static __device__ __forceinline__ double exp2_(double v) { return exp2(v); }
    static __device__ __forceinline__ void normals(double u1, double u2, double &z1, double &z2) {
        const double r = sqrt(-2.0 * log(u1));
        double s, c;
        sincospi(2.0 * u2, &s, &c);
        z1 = r * c;
        z2 = r * s;
    }
    static __device__ __forceinline__ double unit(uint32_t w) { return unit_u24d(w); }
};

// Philox words of step pair `step2` of a path under the path scheme: plain
// (counter (path, step2, 0, 2)), or antithetic pairs, in which paths 2k and
// 2k + 1 both draw counter (k, step2, 0, 2) and the odd path negates the
// normals (path_sign).
__device__ __forceinline__ uint4 path_words(int64_t path, uint32_t step2, bool anti, uint32_t k0, uint32_t k1) {
    return philox4x32_10(make_uint4((uint32_t)(anti ? (path >> 1) : path), step2, 0u, 2u), k0, k1);
}
template <typename R>
__device__ __forceinline__ R path_sign(int64_t path, bool anti) {
    return (anti && (path & 1)) ? (R)-1 : (R)1;
}

// Functional parameters of the three models at time t (eqs. "el_fun_1",
// "el_fun_3"); the static model has constant nu, rho.
template <typename R>
__device__ __forceinline__ void nu_rho_at(int model, const double *x, double t, double &nu, double &rho) {
    if (model == MODEL_STATIC) {
        nu = x[2];
        rho = x[1];
    } else if (model == MODEL_DYN_I) {
        nu = x[2] * exp(-x[4] * t);
        rho = x[1] * exp(-x[3] * t);
    } else {
        nu = fma(x[8], t, x[2]) * exp(-x[4] * t) + x[6];
        rho = fma(x[7], t, x[1]) * exp(-x[3] * t) + x[5];
    }
}

// Step coefficients of one parameter set: {nu sqrt(dt)/ln2, -nu^2 dt/(2 ln2),
// rho sqrt(dt)/ln2, sqrt(1-rho^2) sqrt(dt)/ln2} at t = s dt (left point).
template <typename R>
struct StepC {
    R nz, nd, rz, rp;
};
template <typename R>
__device__ __forceinline__ StepC<R> step_coeffs(int model, const double *x, double t, double dt) {
    double nu, rho;
    nu_rho_at<R>(model, x, t, nu, rho);
    const double sdt = sqrt(dt) / kLn2;
    StepC<R> c;
    c.nz = (R)(nu * sdt);
    c.nd = (R)(-nu * nu * dt / (2.0 * kLn2));
    c.rz = (R)(rho * sdt);
    c.rp = (R)(sqrt(fmax(1.0 - rho * rho, 0.0)) * sdt);
    return c;
}

__device__ __forceinline__ float bcast(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

__device__ __forceinline__ double mc_propose(double x, double u, double h, double lb, double ub) {
#pragma clang fp contract(off)
    double y = x + (h * (2.0 * u - 1.0)) * (ub - lb);
    if (y > ub) y = ub - (y - ub);
    if (y < lb) y = lb + (lb - y);
    if (y > ub) y = ub;
    if (y < lb) y = lb;
    return y;
}

// Step coefficients at time t in float, from float parameters (the Monte
// Carlo objective of the dynamic models evaluates them every step).
template <int MODEL>
__device__ __forceinline__ StepC<float> step_coeffs_f(const float *xf, float t, float sdt, float ndt) {
    constexpr float kLog2e = 1.4426950408889634f;
    float nu, rho;
    if constexpr (MODEL == MODEL_DYN_I) {
        nu = xf[2] * __builtin_amdgcn_exp2f(-xf[4] * t * kLog2e);
        rho = xf[1] * __builtin_amdgcn_exp2f(-xf[3] * t * kLog2e);
    } else {
        nu = fmaf(xf[8], t, xf[2]) * __builtin_amdgcn_exp2f(-xf[4] * t * kLog2e) + xf[6];
        rho = fmaf(xf[7], t, xf[1]) * __builtin_amdgcn_exp2f(-xf[3] * t * kLog2e) + xf[5];
    }
    StepC<float> c;
    c.nz = nu * sdt;
    c.nd = nu * nu * ndt;
    c.rz = rho * sdt;
    c.rp = __builtin_amdgcn_sqrtf(fmaxf(1.0f - rho * rho, 0.0f)) * sdt;
    return c;
}

// Common-random-number pricing of one wave: lane = one parameter vector of
// the tile, the wave walks the paths [pb * ppb, (pb + 1) * ppb) NPATH at a
// time so that every lane carries NPATH independent recurrences.  The
// normals of a step are made once per wave (lane q * LPP + j draws the
// Philox block (path q, step pair j) and turns both of its pairs into
// normals) and broadcast to all lanes; payoffs go to per-lane float sums in
// LDS, one per option (ACC_LDS).  ACC_DIRECT: the block is one round of
// NPATH paths, so each option's sum over them is complete at its maturity and
// goes straight to the partials in HBM.  ACC_HBM: the block's rounds add
// into the block's own partials in HBM (each lane its own words).  Both
// leave LDS free of the per-option sums, which otherwise set the occupancy
// (n_obs x 64 floats per wave).
// With LDSB the normals of a chunk go through a small LDS table (one
// broadcast read per step and path) instead of lane reads into scalar
// registers.
constexpr int kCrnPaths = 16;       // paths per lane of the production kernels
constexpr bool kCrnLdsNormals = true;
__host__ __device__ constexpr int crn_normals_bytes() { return 1024; }   // NPATH x CH float2 = 128 x 8 B (any NPATH)

enum { ACC_LDS = 0, ACC_DIRECT = 1, ACC_HBM = 2 };
template <int MODEL, int NPATH = kCrnPaths, bool LDSB = kCrnLdsNormals, int ACC = ACC_LDS>
__device__ inline void crn_block(const McCrnDesc &d, int tile, int pb, const double *Y, const int32_t *mat_steps,
                          const int32_t *offs, const double *K, float *part, unsigned char *smem) {
    constexpr int LPP = 64 / NPATH;          // lanes per path when drawing normals
    constexpr int CH = 2 * LPP;              // steps per chunk
    float2 *ztab = reinterpret_cast<float2 *>(smem);  // [NPATH][CH] normals (LDSB), 1 KB
    float *Ks = reinterpret_cast<float *>(smem + crn_normals_bytes());
    float *acc = Ks + ((d.n_obs + 3) / 4) * 4;        // [n_obs][64]
    const int lane = threadIdx.x;
    for (int o = lane; o < d.n_obs; o += 64) Ks[o] = (float)K[o];
    if constexpr (ACC == ACC_LDS)
        for (int o = 0; o < d.n_obs; ++o) acc[o * 64 + lane] = 0.0f;
    const int64_t chain = (int64_t)tile * 64 + lane;
    const bool active = chain < d.n_chains;
    constexpr int NP = MODEL == MODEL_STATIC ? 3 : (MODEL == MODEL_DYN_I ? 5 : 9);
    double x[NP];
    float xf[NP];
    for (int k = 0; k < NP; ++k) {
        x[k] = active ? Y[chain * d.np_stride + k] : (k == 0 ? 0.2 : 0.0);
        xf[k] = (float)x[k];
    }
    const double beta = d.beta_free ? (active ? Y[chain * d.np_stride + NP] : 1.0) : d.beta;
    const float bm1 = (float)(beta - 1.0);
    const float hd = (float)(d.dt / (2.0 * kLn2));
    const float xabs = (float)kLog2Abs;
    const float A0 = (float)(log2(x[0]) + (beta - 1.0) * log2(d.f0));
    const StepC<float> cst = step_coeffs<float>(MODEL_STATIC, x, 0.0, d.dt);
    const float sdt = (float)(sqrt(d.dt) / kLn2), ndt = (float)(-d.dt / (2.0 * kLn2)), dtf = (float)d.dt;
    const float f0 = (float)d.f0;
    const int q_self = lane / LPP, j_self = lane % LPP;
    __syncthreads();
    const int64_t p_begin = (int64_t)pb * d.paths_per_block;
    const int64_t p_end = min<int64_t>(p_begin + d.paths_per_block, d.n_paths);
    if constexpr (ACC != ACC_LDS) {
        // a block past the last path still owns its (zero) partial sums
        if (p_begin >= p_end) {
            for (int o = 0; o < d.n_obs; ++o) part[(((size_t)tile * d.n_obs + o) * d.n_pblocks + pb) * 64 + lane] = 0.0f;
            return;
        }
    }
    for (int64_t path = p_begin; path < p_end; path += NPATH) {
        const int n_live = (int)min<int64_t>(NPATH, p_end - path);
        // X: log2(F/f0), -inf once absorbed; Xc: X clamped at the absorption
        // level (what the local volatility sees, finite)
        float X[NPATH], Xc[NPATH], A[NPATH];
#pragma unroll
        for (int q = 0; q < NPATH; ++q) {
            X[q] = 0.0f;
            Xc[q] = 0.0f;
            A[q] = A0;
        }
        int mi = 0;
        int mnext = mat_steps[0];
        for (int s0 = 0; s0 < d.m_max; s0 += CH) {
            const uint4 w = path_words(path + q_self, (uint32_t)((s0 >> 1) + j_self), d.anti != 0, d.key0, d.key1);
            float ze1, ze2, zo1, zo2;
            MC<float>::normals(unit_u24f(w.x), unit_u24f(w.y), ze1, ze2);
            MC<float>::normals(unit_u24f(w.z), unit_u24f(w.w), zo1, zo2);
            if (d.anti && ((path + q_self) & 1)) {
                ze1 = -ze1;
                ze2 = -ze2;
                zo1 = -zo1;
                zo2 = -zo2;
            }
            if constexpr (LDSB) {
                __syncthreads();
                ztab[(2 * j_self) * NPATH + q_self] = make_float2(ze1, ze2);
                ztab[(2 * j_self + 1) * NPATH + q_self] = make_float2(zo1, zo2);
                __syncthreads();
            }
            const int n_here = min(CH, d.m_max - s0);
#pragma unroll
            for (int l = 0; l < CH; ++l) {
                if (l < n_here) {
                    StepC<float> c = cst;
                    if constexpr (MODEL != MODEL_STATIC) c = step_coeffs_f<MODEL>(xf, (float)(s0 + l) * dtf, sdt, ndt);
                    // the step's normals of all paths first (one LDS wait per step)
                    float2 zz[NPATH];
#pragma unroll
                    for (int q = 0; q < NPATH; ++q) {
                        if constexpr (LDSB) {
                            zz[q] = ztab[l * NPATH + q];
                        } else {
                            const int src = q * LPP + (l >> 1);
                            zz[q] = make_float2(bcast((l & 1) ? zo1 : ze1, src), bcast((l & 1) ? zo2 : ze2, src));
                        }
                    }
#pragma unroll
                    for (int q = 0; q < NPATH; ++q) {
                        const float z1 = zz[q].x, z2 = zz[q].y;
                        const float vh = __builtin_amdgcn_exp2f(fmaf(bm1, Xc[q], A[q]));
                        A[q] = fmaf(c.nz, z1, A[q] + c.nd);
                        const float w2 = fmaf(c.rz, z1, c.rp * z2);
                        const float Xn = fmaf(vh, fmaf(-hd, vh, w2), X[q]);
                        const bool absorbed = Xn < xabs;
                        X[q] = absorbed ? -__builtin_inff() : Xn;
                        Xc[q] = absorbed ? xabs : Xn;
                    }
                    if (s0 + l + 1 == mnext) {
                        float F[NPATH];
#pragma unroll
                        for (int q = 0; q < NPATH; ++q) F[q] = q < n_live ? f0 * __builtin_amdgcn_exp2f(X[q]) : 0.0f;
                        do {
                            for (int o = offs[mi]; o < offs[mi + 1]; ++o) {
                                float pay = 0.0f;
#pragma unroll
                                for (int q = 0; q < NPATH; ++q) pay += fmaxf(F[q] - Ks[o], 0.0f);
                                if constexpr (ACC == ACC_LDS) {
                                    acc[o * 64 + lane] += pay;
                                } else {
                                    float *pp = part + (((size_t)tile * d.n_obs + o) * d.n_pblocks + pb) * 64 + lane;
                                    *pp = (ACC == ACC_HBM && path != p_begin) ? *pp + pay : pay;
                                }
                            }
                            ++mi;
                            mnext = mi < d.n_mat ? mat_steps[mi] : -1;
                        } while (mnext == s0 + l + 1);
                    }
                }
            }
        }
    }
    // partial layout: [tile][obs][pblock][lane]
    if constexpr (ACC == ACC_LDS)
        for (int o = 0; o < d.n_obs; ++o)
            part[(((size_t)tile * d.n_obs + o) * d.n_pblocks + pb) * 64 + lane] = acc[o * 64 + lane];
}

// Price of option o for the 64 chains of one tile from the path-block
// partial sums, by a block of 256 threads (four waves): wave w adds the
// blocks w, w + 4, ... in double, the four wave sums are added in order.
// price = disc * S / N; e2[o][chain] = ((target - price) sw)^2, +inf for a
// price that is not finite.
__device__ inline void crn_price_tile(const McCrnDesc &d, int tile, int o, const float *part, const int32_t *obs_row,
                                      const double *disc, const double *target, const double *sw, double *model,
                                      double *e2, int64_t e2_stride, double *s_sum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const float *p = part + (((size_t)tile * d.n_obs + o) * d.n_pblocks) * 64 + lane;
    // four blocks' partials read together into four sums (four loads in
    // flight per wave), then the rest
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = w;
    for (; b + 3 * nw < d.n_pblocks; b += 4 * nw) {
        const float v0 = p[(size_t)b * 64], v1 = p[(size_t)(b + nw) * 64];
        const float v2 = p[(size_t)(b + 2 * nw) * 64], v3 = p[(size_t)(b + 3 * nw) * 64];
        s0 += (double)v0;
        s1 += (double)v1;
        s2 += (double)v2;
        s3 += (double)v3;
    }
    for (; b < d.n_pblocks; b += nw) s0 += (double)p[(size_t)b * 64];
    s_sum[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    const int64_t chain = (int64_t)tile * 64 + lane;
    if (w == 0 && chain < d.n_chains) {
        double tot = s_sum[lane];
        for (int k = 1; k < nw; ++k) tot += s_sum[k * 64 + lane];
        const double price = disc[obs_row[o]] * tot * (1.0 / (double)d.n_paths);
        const bool ok = price > -__builtin_inf() && price < __builtin_inf();
        if (model) model[chain * d.n_obs + o] = price;
        if (e2) {
            const double e = (target[o] - price) * sw[o];
            e2[(int64_t)o * e2_stride + chain] = ok ? e * e : __builtin_inf();
        }
    }
}

// f of one chain: the squared errors added over the options in order; an
// infeasible case II vector gives +inf.
__device__ inline double crn_chain_objective(const McCrnDesc &d, int64_t chain, const double *Y, const double *e2,
                                             int64_t e2_stride) {
    double f = 0.0;
    for (int o = 0; o < d.n_obs; ++o) f += e2[(int64_t)o * e2_stride + chain];
    if (d.model == MODEL_DYN_II && !case2_feasible(Y + chain * d.np_stride, d.t_max)) f = __builtin_inf();
    return f;
}

__device__ inline void mc_step_body(const McSaDesc &d, int t, const double *sched_g, const double *sched_h,
                             const double *fy, double *Y, McSaState *stp, double *cx, double *cf, double *bx,
                             double *bf, double *s_f, int *s_id) {
    McSaState &st = *stp;
    const int NP = d.n_par;
    const int P = d.n_chains;
    const int L = d.chain_len;
    if (t < 0) {
        const double f0 = (fy[0] == fy[0]) ? fy[0] : __builtin_inf();
        if (threadIdx.x == 0) {
            st.T0 = d.T0 > 0.0 ? d.T0 : ((f0 > 0.0 && f0 < __builtin_inf()) ? f0 : 1.0);
            st.n_accept = 0;
        }
        for (int c = threadIdx.x; c < P; c += blockDim.x) {
            for (int k = 0; k < NP; ++k) cx[c * NP + k] = bx[c * NP + k] = d.x0[k];
            cf[c] = bf[c] = f0;
        }
    } else {
        const int lev = t / L;
        const double Tk = st.T0 * sched_g[lev];
        const int nb = (NP + 1 + 3) / 4;
        unsigned long long nacc = 0;
        for (int c = threadIdx.x; c < P; c += blockDim.x) {
            const int b = NP / 4;
            const uint4 w = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)t, (uint32_t)b, 1u), d.key0, d.key1);
            const uint32_t words[4] = {w.x, w.y, w.z, w.w};
            const double ua = unit_u32(words[NP % 4]);
            (void)nb;
            double v = fy[c];
            if (!(v == v)) v = __builtin_inf();
            if (d.model == MODEL_DYN_II && !case2_feasible(Y + (size_t)c * NP, d.t_max)) v = __builtin_inf();
            const double delta = v - cf[c];
            bool acc;
            {
#pragma clang fp contract(off)
                acc = delta <= 0.0 || ua < exp(-delta / Tk);
            }
            if (acc) {
                for (int k = 0; k < NP; ++k) cx[c * NP + k] = Y[(size_t)c * NP + k];
                cf[c] = v;
                ++nacc;
                if (v < bf[c]) {
                    bf[c] = v;
                    for (int k = 0; k < NP; ++k) bx[c * NP + k] = Y[(size_t)c * NP + k];
                }
            }
        }
        __syncthreads();
        // count accepted moves
        s_id[threadIdx.x] = (int)nacc;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long tot = 0;
            for (int i = 0; i < (int)blockDim.x; ++i) tot += (unsigned long long)s_id[i];
            st.n_accept += tot;
        }
        __syncthreads();
        const bool level_end = ((t + 1) % L == 0) || (t + 1 == d.n_iters);
        if (level_end) {
            double f = __builtin_inf();
            int id = 0x7fffffff;
            for (int c = threadIdx.x; c < P; c += blockDim.x)
                if (cf[c] < f || (cf[c] == f && c < id)) {
                    f = cf[c];
                    id = c;
                }
            s_f[threadIdx.x] = f;
            s_id[threadIdx.x] = id;
            __syncthreads();
            if (threadIdx.x == 0) {
                double bfv = s_f[0];
                int bid = s_id[0];
                for (int i = 1; i < (int)blockDim.x; ++i)
                    if (s_f[i] < bfv || (s_f[i] == bfv && s_id[i] < bid)) {
                        bfv = s_f[i];
                        bid = s_id[i];
                    }
                s_f[0] = bfv;
                s_id[0] = bid;
            }
            __syncthreads();
            const int bid = s_id[0];
            const double bfv = s_f[0];
            if (bid < P) {
                double xb[kMaxPar];
                for (int k = 0; k < NP; ++k) xb[k] = cx[bid * NP + k];
                __syncthreads();
                for (int c = threadIdx.x; c < P; c += blockDim.x) {
                    for (int k = 0; k < NP; ++k) cx[c * NP + k] = xb[k];
                    cf[c] = bfv;
                }
            }
        }
    }
    __syncthreads();
    // proposals of iteration t + 1
    const int tn = t + 1;
    if (tn < d.n_iters) {
        const int lev = tn / L;
        const double h = sched_h[lev];
        for (int c = threadIdx.x; c < P; c += blockDim.x) {
            double u[12];
            for (int b = 0; b * 4 < NP + 1; ++b) {
                const uint4 w = philox4x32_10(make_uint4((uint32_t)c, (uint32_t)tn, (uint32_t)b, 1u), d.key0, d.key1);
                u[4 * b + 0] = unit_u32(w.x);
                u[4 * b + 1] = unit_u32(w.y);
                u[4 * b + 2] = unit_u32(w.z);
                u[4 * b + 3] = unit_u32(w.w);
            }
            for (int k = 0; k < NP; ++k)
                Y[(size_t)c * NP + k] = mc_propose(cx[c * NP + k], u[k], h, d.lb[k], d.ub[k]);
        }
    }
}

// Final best over the chains (lowest index on ties).
__device__ inline void mc_final_body(const McSaDesc &d, const double *bx, const double *bf, McSaState *st) {
    int best = 0;
    for (int c = 1; c < d.n_chains; ++c)
        if (bf[c] < bf[best]) best = c;
    st->best_f = bf[best];
    for (int k = 0; k < d.n_par; ++k) st->best_x[k] = bx[best * d.n_par + k];
}

}  // namespace sabr
