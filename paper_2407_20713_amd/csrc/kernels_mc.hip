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
#include "sabr_mc.h"

namespace sabr {

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
        const bool anti = d.anti != 0;
        const R sg = path_sign<R>(path, anti);
        R X = 0, A = A0;
        int mi = 0;
        uint4 w = make_uint4(0, 0, 0, 0);
        for (int s = 0; s < d.m_max; ++s) {
            if ((s & 1) == 0) w = path_words(path, (uint32_t)(s >> 1), anti, d.key0, d.key1);
            const R u1 = MC<R>::unit((s & 1) ? w.z : w.x);
            const R u2 = MC<R>::unit((s & 1) ? w.w : w.y);
            R z1, z2;
            MC<R>::normals(u1, u2, z1, z2);
            z1 *= sg;
            z2 *= sg;
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
                    // antithetic: one squared sample per pair (its mean, on the
                    // even lane); a pair is two neighbouring lanes
                    double vs = v, vq = v * v;
                    if (anti) {   // uniform over the launch
                        const double pm = 0.5 * (v + __shfl_xor(v, 1, 64));
                        vq = (lane & 1) ? 0.0 : pm * pm;
                    }
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

// Path grid of a Monte Carlo pricing call from the raw grid in device
// memory: step of each maturity max(1, floor(T dt^-1 + 1e-9)) (the host's
// rule, in the same double arithmetic), maturity row of each option, and the
// discount factors (1 where none are given).  One thread per option.
__global__ void mc_grid_kernel(int n_mat, const double *T, const int32_t *offs, int spy, const double *disc_in,
                               int32_t *msteps, int32_t *obsrow, double *disc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n_mat) {
        const int m = (int)floor(T[j] * (double)spy + 1e-9);
        msteps[j] = m < 1 ? 1 : m;
        disc[j] = disc_in ? disc_in[j] : 1.0;
    }
    if (j < offs[n_mat]) {
        int i = 0;
        while (offs[i + 1] <= j) ++i;
        obsrow[j] = i;
    }
}

// Sums of the workgroup partials in a fixed order: price = disc * S / N and
// its standard error.
__global__ void mc_price_finalize(int n_obs, int n_blocks, int64_t n_paths, int anti, const double *part_s,
                                  const double *part_q, const int32_t *obs_row, const double *disc,
                                  double *price, double *se) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obs) return;
    double s = 0.0, q = 0.0;
    for (int b = 0; b < n_blocks; ++b) {
        s += part_s[(size_t)b * n_obs + o];
        q += part_q[(size_t)b * n_obs + o];
    }
    // samples: the paths, or the antithetic pairs (q then sums the squared
    // pair means; their mean is the mean over all paths)
    const int64_t n_samp = anti ? n_paths / 2 : n_paths;
    const double N = (double)n_samp;
    const double mean = s / (double)n_paths;
    const double var = n_samp > 1 ? fmax(q / N - mean * mean, 0.0) * N / (N - 1.0) : 0.0;
    const double D = disc[obs_row[o]];
    price[o] = D * mean;
    se[o] = D * sqrt(var / N);
}

// ---------------------------------------------------------------------------
// Cliquet (Section 6, eqs. "eq_cliquet" and "eq:cliquet_global") on the paths
// of the pricing kernel above, one parameter set: lane = path.  The forward
// is read at the reset dates d_1 < ... < d_D (step max(1, floor(d_i / dt)),
// as for the European maturities); each return R_i = (F_{d_i} - F_{d_{i-1}}) /
// F_{d_{i-1}}, i = 2..D, is clamped to [local floor, local cap] and the
// returns are summed; the sum is clamped to [global floor, global cap] (the
// printed max/min of the global payoff read so that the floor is the lower
// limit).  A return from an absorbed (zero) forward is -1.  Payoffs and their
// squares are summed over the wave in double and per wave in LDS; the
// workgroup writes its two sums once, and mc_price_finalize turns them into
// the discounted mean and its standard error.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void __launch_bounds__(256) mc_cliquet_kernel(CliqDesc d, const int32_t *reset_steps, double *part_s,
                                                        double *part_q) {
    extern __shared__ unsigned char smem[];
    StepC<R> *st = reinterpret_cast<StepC<R> *>(smem);
    double *acc_s = reinterpret_cast<double *>(smem + sizeof(StepC<R>) * ((d.m_max + 1) / 2 * 2));
    double *acc_q = acc_s + 4;
    for (int s = threadIdx.x; s < d.m_max; s += blockDim.x) st[s] = step_coeffs<R>(d.model, d.x, s * d.dt, d.dt);
    if (threadIdx.x < 4) acc_s[threadIdx.x] = acc_q[threadIdx.x] = 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const R bm1 = (R)(d.beta - 1.0);
    const R hd = (R)(d.dt / (2.0 * kLn2));
    const R xabs = (R)kLog2Abs;
    const R A0 = (R)(log2(d.x[0]) + (d.beta - 1.0) * log2(d.f0));
    const R f0 = (R)d.f0;
    const R lf = (R)d.local_floor, lc = (R)d.local_cap, gf = (R)d.global_floor, gc = (R)d.global_cap;
    const int64_t n_tiles = (d.n_paths + 255) / 256;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t path = tile * 256 + threadIdx.x;
        const bool active = path < d.n_paths;
        const bool anti = d.anti != 0;
        const R sg = path_sign<R>(path, anti);
        R X = 0, A = A0, Fp = 0, sum = 0;
        int next = 0;
        uint4 w = make_uint4(0, 0, 0, 0);
        for (int s = 0; s < d.m_max; ++s) {
            if ((s & 1) == 0) w = path_words(path, (uint32_t)(s >> 1), anti, d.key0, d.key1);
            const R u1 = MC<R>::unit((s & 1) ? w.z : w.x);
            const R u2 = MC<R>::unit((s & 1) ? w.w : w.y);
            R z1, z2;
            MC<R>::normals(u1, u2, z1, z2);
            z1 *= sg;
            z2 *= sg;
            const StepC<R> c = st[s];
            const R vh = MC<R>::exp2_(fma(bm1, fmax(X, xabs), A));
            A = fma(c.nz, z1, A + c.nd);
            const R w2 = fma(c.rz, z1, c.rp * z2);
            const R Xn = fma(vh, fma(-hd, vh, w2), X);
            X = (Xn < xabs) ? -(R)__builtin_inff() : Xn;
            if (next < d.n_reset && reset_steps[next] == s + 1) {
                const R F = f0 * MC<R>::exp2_(X);
                if (next > 0) {
                    const R ret = Fp > (R)0 ? (F - Fp) / Fp : (R)-1;
                    sum += fmax(fmin(ret, lc), lf);
                }
                Fp = F;
                ++next;
            }
        }
        const double v = active ? (double)fmax(gf, fmin(gc, sum)) : 0.0;
        double vs = v, vq = v * v;
        if (anti) {   // one squared sample per antithetic pair (neighbouring lanes), on the even lane
            const double pm = 0.5 * (v + __shfl_xor(v, 1, 64));
            vq = (lane & 1) ? 0.0 : pm * pm;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            vs += __shfl_xor(vs, off, 64);
            vq += __shfl_xor(vq, off, 64);
        }
        if (lane == 0) {
            acc_s[wave] += vs;
            acc_q[wave] += vq;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0, q = 0.0;
        for (int wv = 0; wv < 4; ++wv) {
            s += acc_s[wv];
            q += acc_q[wv];
        }
        part_s[blockIdx.x] = s;
        part_q[blockIdx.x] = q;
    }
}

// ---------------------------------------------------------------------------
// Common-random-number kernel for the Monte Carlo objective: lane = one
// parameter set (chain), a whole wave follows the same path.  The normals of
// 64 steps are drawn cooperatively (lane l draws step s0 + l) and broadcast
// with readlane, so each (path, step) costs one Philox half and one
// Box-Muller for 64 chains.  Payoffs are summed per lane in LDS in float over
// the paths of the block; partial sums go to device memory lane-contiguous.
// ---------------------------------------------------------------------------
template <int MODEL, int NPATH, bool LDSB, int ACC = ACC_LDS>
__global__ void __launch_bounds__(64) mc_crn_kernel(McCrnDesc d, const double *Y, const int32_t *mat_steps,
                                                   const int32_t *offs, const double *K, float *part) {
    extern __shared__ unsigned char smem[];
    crn_block<MODEL, NPATH, LDSB, ACC>(d, blockIdx.x / d.n_pblocks, blockIdx.x % d.n_pblocks, Y, mat_steps, offs,
                                          K, part, smem);
}

// Model prices and squared errors: grid (tiles, options), 256 threads.
__global__ void __launch_bounds__(256) mc_crn_prices(McCrnDesc d, const float *part, const int32_t *obs_row,
                                                    const double *disc, const double *target, const double *sw,
                                                    double *model, double *e2, int64_t e2_stride) {
    __shared__ double s_sum[256];
    crn_price_tile(d, blockIdx.x, blockIdx.y, part, obs_row, disc, target, sw, model, e2, e2_stride, s_sum);
}

// Objective per chain from the squared errors.
__global__ void __launch_bounds__(256) mc_crn_objective(McCrnDesc d, const double *Y, const double *e2,
                                                       int64_t e2_stride, double *f) {
    const int64_t chain = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (chain < d.n_chains) f[chain] = crn_chain_objective(d, chain, Y, e2, e2_stride);
}

// ---------------------------------------------------------------------------
// Annealing step for the Monte Carlo objective (Technique II, with the chains
// kept on the device): one workgroup per request.  Step t accepts or rejects
// the proposals of iteration t whose objectives fy[] were just computed, ends
// the level when t closes one (argmin over current states, every chain
// restarts from it), and proposes iteration t + 1.  t = -1 initialises every
// chain at x0 with fy[0] = f(x0).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(1024) mc_sa_step(McSaDesc d, int t, const double *sched_g,
                                                  const double *sched_h, const double *fy, double *Y,
                                                  McSaState *stp, double *cx, double *cf, double *bx,
                                                  double *bf) {
    __shared__ double s_f[1024];
    __shared__ int s_id[1024];
    mc_step_body(d, t, sched_g, sched_h, fy, Y, stp, cx, cf, bx, bf, s_f, s_id);
}

__global__ void mc_sa_final(McSaDesc d, const double *bx, const double *bf, McSaState *st) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    mc_final_body(d, bx, bf, st);
}

// ---------------------------------------------------------------------------
const void *mc_price_kernel_ptr(bool fp32) {
    return fp32 ? (const void *)mc_price_kernel<float> : (const void *)mc_price_kernel<double>;
}
const void *mc_price_finalize_ptr() { return (const void *)mc_price_finalize; }
const void *mc_grid_kernel_ptr() { return (const void *)mc_grid_kernel; }
const void *mc_cliquet_kernel_ptr(bool fp32) {
    return fp32 ? (const void *)mc_cliquet_kernel<float> : (const void *)mc_cliquet_kernel<double>;
}
size_t mc_cliquet_smem_bytes(bool fp32, int m_max) {
    const size_t st = (fp32 ? sizeof(StepC<float>) : sizeof(StepC<double>)) * (size_t)((m_max + 1) / 2 * 2);
    return st + 8 * sizeof(double);
}
// variant: 0 = the production layout (kCrnPaths, kCrnLdsNormals); 1..8 =
// (1, 2, 4, 8 paths per lane) x (scalar broadcast, LDS broadcast); 9 = 16
// paths per lane with LDS broadcast; for tuning.
const void *mc_crn_kernel_ptr(int model, int variant) {
#define SABR_CRN(MD)                                                                                           \
    {(const void *)mc_crn_kernel<MD, kCrnPaths, kCrnLdsNormals>, (const void *)mc_crn_kernel<MD, 1, false>,      \
     (const void *)mc_crn_kernel<MD, 2, false>, (const void *)mc_crn_kernel<MD, 4, false>,                       \
     (const void *)mc_crn_kernel<MD, 8, false>, (const void *)mc_crn_kernel<MD, 1, true>,                        \
     (const void *)mc_crn_kernel<MD, 2, true>, (const void *)mc_crn_kernel<MD, 4, true>,                         \
     (const void *)mc_crn_kernel<MD, 8, true>, (const void *)mc_crn_kernel<MD, 16, true>}
    static const void *tab[3][10] = {SABR_CRN(MODEL_STATIC), SABR_CRN(MODEL_DYN_I), SABR_CRN(MODEL_DYN_II)};
#undef SABR_CRN
    if (model < 0 || model > 2 || variant < 0 || variant > 9) return nullptr;
    return tab[model][variant];
}
// one round of kCrnPaths paths per block, sums straight to HBM
const void *mc_crn_direct_kernel_ptr(int model) {
    static const void *tab[3] = {(const void *)mc_crn_kernel<MODEL_STATIC, kCrnPaths, kCrnLdsNormals, ACC_DIRECT>,
                                 (const void *)mc_crn_kernel<MODEL_DYN_I, kCrnPaths, kCrnLdsNormals, ACC_DIRECT>,
                                 (const void *)mc_crn_kernel<MODEL_DYN_II, kCrnPaths, kCrnLdsNormals, ACC_DIRECT>};
    return (model < 0 || model > 2) ? nullptr : tab[model];
}
int mc_crn_direct_paths() { return kCrnPaths; }
const void *mc_crn_prices_ptr() { return (const void *)mc_crn_prices; }
const void *mc_crn_objective_ptr() { return (const void *)mc_crn_objective; }
const void *mc_sa_step_ptr() { return (const void *)mc_sa_step; }
const void *mc_sa_final_ptr() { return (const void *)mc_sa_final; }
size_t mc_price_smem_bytes(bool fp32, int m_max, int n_obs) {
    const size_t rs = fp32 ? sizeof(float) : sizeof(double);
    const size_t st = (fp32 ? sizeof(StepC<float>) : sizeof(StepC<double>)) * m_max;
    return st + (rs * n_obs + 15) / 16 * 16 + 2 * 4 * sizeof(double) * n_obs;
}
size_t mc_crn_smem_bytes(int n_obs, bool direct) {
    return crn_normals_bytes() + sizeof(float) * (((n_obs + 3) / 4) * 4 + (direct ? 0 : 64 * (size_t)n_obs));
}

}  // namespace sabr
