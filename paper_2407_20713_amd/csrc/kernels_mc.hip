// kernels_mc.hip -- Monte Carlo pricing by the log-Euler scheme of Section 4
// (eq. "dis_SABRd", estimator eq. "payoff").
//
// The state of a path is kept in base-2 logarithms so that one v_exp_f32 per
// step gives the local vol: X = log2(F / F0), A = log2(alpha) + (beta - 1)
// log2(F0), so that nuhat = alpha F^(beta-1) = 2^(A + (beta - 1) X).  A step
// of the printed multiplicative scheme is then
//   A += (nu Z1 sqrt(dt) - nu^2 dt / 2) / ln 2
//   X += nuhat ((rho Z1 + sqrt(1 - rho^2) Z2) sqrt(dt) / ln 2 - nuhat dt / (2 ln 2)),
// which is the same recursion.  A forward below 1e-30 F0 is absorbed at 0.
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

// ---------------------------------------------------------------------------
// Pricing kernel, one parameter set: lane = path.  Per-step coefficients,
// strikes and maturity steps are staged in LDS; payoffs of each maturity are
// summed over the wave in double and kept per wave in LDS; the workgroup
// writes its sums (and sums of squares) once.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) mc_price_kernel(McDesc d, const int32_t *mat_steps,
                                                      const int32_t *offs, const double *K,
                                                      double *part_s, double *part_q) {
    extern __shared__ unsigned char smem[];
    StepC<R> *st = reinterpret_cast<StepC<R> *>(smem);
    R *Ks = reinterpret_cast<R *>(smem + sizeof(StepC<R>) * d.m_max);
    const size_t kbytes = (sizeof(R) * d.n_obs + 15) / 16 * 16;
    double *acc_s = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(Ks) + kbytes);
    double *acc_q = acc_s + 4 * d.n_obs;
    for (int s = threadIdx.x; s < d.m_max; s += blockDim.x) st[s] = step_coeffs<R>(d.model, d.x, s * d.dt, d.dt);
    for (int o = threadIdx.x; o < d.n_obs; o += blockDim.x) Ks[o] = (R)K[o];
    for (int o = threadIdx.x; o < 4 * d.n_obs; o += blockDim.x) acc_s[o] = acc_q[o] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const R bm1 = (R)(d.beta - 1.0);
    const R hd = (R)(d.dt / (2.0 * kLn2));
    const R xabs = (R)kLog2Abs;
    const R A0 = (R)(log2(d.x[0]) + (d.beta - 1.0) * log2(d.f0));
    const R f0 = (R)d.f0;
    const int64_t n_tiles = (d.n_paths + 255) / 256;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t path = tile * 256 + threadIdx.x;
        const bool active = path < d.n_paths;
        R X = 0, A = A0;
        int mi = 0;
        uint4 w = make_uint4(0, 0, 0, 0);
        for (int s = 0; s < d.m_max; ++s) {
            if ((s & 1) == 0) w = philox4x32_10(make_uint4((uint32_t)path, (uint32_t)(s >> 1), 0u, 2u), d.key0, d.key1);
            const R u1 = MC<R>::unit((s & 1) ? w.z : w.x);
            const R u2 = MC<R>::unit((s & 1) ? w.w : w.y);
            R z1, z2;
            MC<R>::normals(u1, u2, z1, z2);
            const StepC<R> c = st[s];
            const R vh = MC<R>::exp2_(fma(bm1, fmax(X, xabs), A));
            A = fma(c.nz, z1, A + c.nd);
            const R w2 = fma(c.rz, z1, c.rp * z2);
            const R Xn = fma(vh, fma(-hd, vh, w2), X);
            X = (Xn < xabs) ? -(R)__builtin_inff() : Xn;
            while (mi < d.n_mat && mat_steps[mi] == s + 1) {
                const R F = f0 * MC<R>::exp2_(X);
                for (int o = offs[mi]; o < offs[mi + 1]; ++o) {
                    const double v = active ? (double)fmax(F - Ks[o], (R)0) : 0.0;
                    double vs = v, vq = v * v;
#pragma unroll
                    for (int off = 32; off > 0; off >>= 1) {
                        vs += __shfl_xor(vs, off, 64);
                        vq += __shfl_xor(vq, off, 64);
                    }
                    if (lane == 0) {
                        acc_s[wave * d.n_obs + o] += vs;
                        acc_q[wave * d.n_obs + o] += vq;
                    }
                }
                ++mi;
            }
        }
    }
    __syncthreads();
    for (int o = threadIdx.x; o < d.n_obs; o += blockDim.x) {
        double s = 0.0, q = 0.0;
        for (int wv = 0; wv < 4; ++wv) {
            s += acc_s[wv * d.n_obs + o];
            q += acc_q[wv * d.n_obs + o];
        }
        part_s[(size_t)blockIdx.x * d.n_obs + o] = s;
        part_q[(size_t)blockIdx.x * d.n_obs + o] = q;
    }
}

// Sums of the workgroup partials in a fixed order: price = disc * S / N and
// its standard error.
__global__ void mc_price_finalize(int n_obs, int n_blocks, int64_t n_paths, const double *part_s,
                                  const double *part_q, const int32_t *obs_row, const double *disc,
                                  double *price, double *se) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obs) return;
    double s = 0.0, q = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
        s += part_s[(size_t)b * n_obs + o];
        q += part_q[(size_t)b * n_obs + o];
    }
    const double N = (double)n_paths;
    const double mean = s / N;
    const double var = n_paths > 1 ? fmax(q / N - mean * mean, 0.0) * N / (N - 1.0) : 0.0;
    const double D = disc[obs_row[o]];
    price[o] = D * mean;
    se[o] = D * sqrt(var / N);
}

// ---------------------------------------------------------------------------
// Common-random-number kernel for the Monte Carlo objective: lane = one
// parameter set (chain), a whole wave follows the same path.  The normals of
// 64 steps are drawn cooperatively (lane l draws step s0 + l) and broadcast
// with readlane, so each (path, step) costs one Philox half and one
// Box-Muller for 64 chains.  Payoffs are summed per lane in LDS in float over
// the paths of the block; partial sums go to device memory lane-contiguous.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float bcast(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <int MODEL>
__global__ void __launch_bounds__(64) mc_crn_kernel(McCrnDesc d, const double *Y, const int32_t *mat_steps,
                                                   const int32_t *offs, const double *K, float *part) {
    extern __shared__ unsigned char smem[];
    float *Ks = reinterpret_cast<float *>(smem);
    float *acc = Ks + ((d.n_obs + 3) / 4) * 4;        // [n_obs][64]
    const int lane = threadIdx.x;
    const int tile = blockIdx.x / d.n_pblocks;
    const int pb = blockIdx.x % d.n_pblocks;
    for (int o = lane; o < d.n_obs; o += 64) Ks[o] = (float)K[o];
    for (int o = 0; o < d.n_obs; ++o) acc[o * 64 + lane] = 0.0f;
    const int64_t chain = (int64_t)tile * 64 + lane;
    const bool active = chain < d.n_chains;
    constexpr int NP = MODEL == MODEL_STATIC ? 3 : (MODEL == MODEL_DYN_I ? 5 : 9);
    double x[NP];
    for (int k = 0; k < NP; ++k) x[k] = active ? Y[chain * d.np_stride + k] : (k == 0 ? 0.2 : 0.0);
    const double beta = d.beta_free ? (active ? Y[chain * d.np_stride + NP] : 1.0) : d.beta;
    const float bm1 = (float)(beta - 1.0);
    const float hd = (float)(d.dt / (2.0 * kLn2));
    const float xabs = (float)kLog2Abs;
    const float A0 = (float)(log2(x[0]) + (beta - 1.0) * log2(d.f0));
    StepC<float> cst = step_coeffs<float>(MODEL_STATIC, x, 0.0, d.dt);
    const float f0 = (float)d.f0;
    __syncthreads();
    const int64_t p_begin = (int64_t)pb * d.paths_per_block;
    const int64_t p_end = min<int64_t>(p_begin + d.paths_per_block, d.n_paths);
    for (int64_t path = p_begin; path < p_end; ++path) {
        float X = 0.0f, A = A0;
        int mi = 0;
        int mnext = mat_steps[0];
        for (int s0 = 0; s0 < d.m_max; s0 += 64) {
            const int s = s0 + lane;
            const uint4 w = philox4x32_10(make_uint4((uint32_t)path, (uint32_t)(s >> 1), 0u, 2u), d.key0, d.key1);
            float z1l, z2l;
            MC<float>::normals(unit_u24f((s & 1) ? w.z : w.x), unit_u24f((s & 1) ? w.w : w.y), z1l, z2l);
            const int n_here = min(64, d.m_max - s0);
#pragma unroll
            for (int l = 0; l < 64; ++l) {
                if (l < n_here) {
                    const float z1 = bcast(z1l, l), z2 = bcast(z2l, l);
                    StepC<float> c = cst;
                    if (MODEL != MODEL_STATIC) c = step_coeffs<float>(MODEL, x, (double)(s0 + l) * d.dt, d.dt);
                    const float vh = __builtin_amdgcn_exp2f(fmaf(bm1, fmaxf(X, xabs), A));
                    A = fmaf(c.nz, z1, A + c.nd);
                    const float w2 = fmaf(c.rz, z1, c.rp * z2);
                    const float Xn = fmaf(vh, fmaf(-hd, vh, w2), X);
                    X = (Xn < xabs) ? -__builtin_inff() : Xn;
                    if (s0 + l + 1 == mnext) {
                        const float F = f0 * __builtin_amdgcn_exp2f(X);
                        do {
                            for (int o = offs[mi]; o < offs[mi + 1]; ++o)
                                acc[o * 64 + lane] += fmaxf(F - Ks[o], 0.0f);
                            ++mi;
                            mnext = mi < d.n_mat ? mat_steps[mi] : -1;
                        } while (mnext == s0 + l + 1);
                    }
                }
            }
        }
    }
    // partial layout: [tile][obs][pblock][lane]
    for (int o = 0; o < d.n_obs; ++o)
        part[(((size_t)tile * d.n_obs + o) * d.n_pblocks + pb) * 64 + lane] = acc[o * 64 + lane];
}

// Objective of each chain from the partial sums: price_o = disc * S_o / N,
// f = sum ((target - price) * sw)^2, non-finite prices give +inf.
__global__ void mc_crn_reduce(McCrnDesc d, const double *Y, const float *part, const int32_t *obs_row,
                              const double *disc, const double *target, const double *sw, double *f,
                              double *model, int write_f) {
    const int64_t chain = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (chain >= d.n_chains) return;
    const int tile = (int)(chain / 64), lane = (int)(chain % 64);
    double acc = 0.0;
    bool bad = d.model == MODEL_DYN_II && !case2_feasible(Y + chain * d.np_stride, d.t_max);
    const double invN = 1.0 / (double)d.n_paths;
    for (int o = 0; o < d.n_obs; ++o) {
        const float *p = part + (((size_t)tile * d.n_obs + o) * d.n_pblocks) * 64 + lane;
        double s = 0.0;
        for (int b = 0; b < d.n_pblocks; ++b) s += (double)p[(size_t)b * 64];
        const double price = disc[obs_row[o]] * s * invN;
        bad |= !(price > -__builtin_inf() && price < __builtin_inf());
        if (model) model[chain * d.n_obs + o] = price;
        if (target) {
            const double e = (target[o] - price) * sw[o];
            acc = fma(e, e, acc);
        }
    }
    if (write_f) f[chain] = bad ? __builtin_inf() : acc;
}

// ---------------------------------------------------------------------------
// Annealing step for the Monte Carlo objective (Technique II, with the chains
// kept on the device): one workgroup per request.  Step t accepts or rejects
// the proposals of iteration t whose objectives fy[] were just computed, ends
// the level when t closes one (argmin over current states, every chain
// restarts from it), and proposes iteration t + 1.  t = -1 initialises every
// chain at x0 with fy[0] = f(x0).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mc_propose(double x, double u, double h, double lb, double ub) {
#pragma clang fp contract(off)
    double y = x + (h * (2.0 * u - 1.0)) * (ub - lb);
    if (y > ub) y = ub - (y - ub);
    if (y < lb) y = lb + (lb - y);
    if (y > ub) y = ub;
    if (y < lb) y = lb;
    return y;
}

__global__ void __launch_bounds__(1024) mc_sa_step(McSaDesc d, int t, const double *sched_g,
                                                  const double *sched_h, const double *fy, double *Y,
                                                  McSaState *stp, double *cx, double *cf, double *bx,
                                                  double *bf) {
    __shared__ double s_f[1024];
    __shared__ int s_id[1024];
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
__global__ void mc_sa_final(McSaDesc d, const double *bx, const double *bf, McSaState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int best = 0;
    for (int c = 1; c < d.n_chains; ++c)
        if (bf[c] < bf[best]) best = c;
    st->best_f = bf[best];
    for (int k = 0; k < d.n_par; ++k) st->best_x[k] = bx[best * d.n_par + k];
}

// ---------------------------------------------------------------------------
const void *mc_price_kernel_ptr(bool fp32) {
    return fp32 ? (const void *)mc_price_kernel<float> : (const void *)mc_price_kernel<double>;
}
const void *mc_price_finalize_ptr() { return (const void *)mc_price_finalize; }
const void *mc_crn_kernel_ptr(int model) {
    switch (model) {
        case MODEL_STATIC: return (const void *)mc_crn_kernel<MODEL_STATIC>;
        case MODEL_DYN_I: return (const void *)mc_crn_kernel<MODEL_DYN_I>;
        case MODEL_DYN_II: return (const void *)mc_crn_kernel<MODEL_DYN_II>;
    }
    return nullptr;
}
const void *mc_crn_reduce_ptr() { return (const void *)mc_crn_reduce; }
const void *mc_sa_step_ptr() { return (const void *)mc_sa_step; }
const void *mc_sa_final_ptr() { return (const void *)mc_sa_final; }
size_t mc_price_smem_bytes(bool fp32, int m_max, int n_obs) {
    const size_t rs = fp32 ? sizeof(float) : sizeof(double);
    const size_t st = (fp32 ? sizeof(StepC<float>) : sizeof(StepC<double>)) * m_max;
    return st + (rs * n_obs + 15) / 16 * 16 + 2 * 4 * sizeof(double) * n_obs;
}
size_t mc_crn_smem_bytes(int n_obs) { return sizeof(float) * (((n_obs + 3) / 4) * 4 + 64 * (size_t)n_obs); }

}  // namespace sabr
