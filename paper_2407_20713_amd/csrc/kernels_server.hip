// kernels_server.hip -- kernels of the serving loop (continuous batching of
// calibration requests, Section 5 Techniques I and II).  Every kernel runs
// over the whole slot table and skips slots that are not its kind or not in
// the right state, so one captured graph serves any mix of requests.  A
// request's arithmetic depends only on the request (random words are keyed
// by its seed and chain ids, sums run in a fixed order), so its result is the
// same alone and in any mix, and the same for any quantum length.
#include "sabr_mc.h"
#include "sabr_sa.h"
#include "sabr_server_dev.h"

namespace sabr {

__device__ __forceinline__ PointsD slot_points(const SlotDev &s) {
    return PointsD{s.lfk, s.lkf, s.P1, s.Z, s.Q1, s.Q2, s.target, s.sw, s.row};
}
__device__ __forceinline__ MatsD slot_mats(const SlotDev &s) { return MatsD{s.T, s.lnf, s.F1, s.offs}; }

// Grid normalisation of newly admitted formula slots (one workgroup per slot
// of [first, first + gridDim.x)).
__global__ void __launch_bounds__(256) slot_prepare_kernel(SlotDev *slots, int first) {
    SlotDev &s = slots[first + blockIdx.x];
    if (s.state != SLOT_NEW) return;
    if (s.kind != KIND_MC) {
        const ReqDesc &rq = s.rq;
        for (int i = 0; i < rq.n_mat; ++i) {
            const double f = s.fwd[i];
            const double beta = rq.beta_free ? 1.0 : rq.beta;
            for (int j = s.offs[i] + threadIdx.x; j < s.offs[i + 1]; j += blockDim.x) {
                normalise_point(s.K[j], f, beta, rq.formula, rq.weighting, s.target[j], s.lfk[j], s.lkf[j], s.P1[j],
                                s.Z[j], s.Q1[j], s.Q2[j], s.sw[j]);
                s.row[j] = i;
            }
            if (threadIdx.x == 0) {
                s.lnf[i] = log(f);
                s.F1[i] = exp((1.0 - beta) * log(f));
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) s.state = SLOT_READY;
}

// ---------------------------------------------------------------------------
// Annealing quantum of the formula slots: one workgroup per slot advances its
// request by up to Q temperature levels (static: two lanes per chain, up to
// 256 chains; dynamic case I: one lane per chain, up to 512 chains), keeping
// the chain state in HBM between quanta.  On the last level the best state is
// polished by the first wave (double-precision Levenberg-Marquardt).
// ---------------------------------------------------------------------------
template <int KIND>
__device__ void sa_slot_body(SlotDev &s, int Q, unsigned char *smem) {
    constexpr int MODEL = KIND == KIND_STATIC ? MODEL_STATIC : MODEL_DYN_I;
    constexpr int FORMULA = F_HAGAN;
    constexpr int LPC = KIND == KIND_STATIC ? 2 : 1;
    constexpr int NP = base_npar<MODEL>();
    constexpr int NB = (NP + 1 + 3) / 4;
    const ReqDesc &rq = s.rq;
    ArgminSmem &am = *reinterpret_cast<ArgminSmem *>(smem);
    double *s_lb = reinterpret_cast<double *>(smem + sizeof(ArgminSmem));
    double *s_ub = s_lb + kMaxPar;
    unsigned char *grid = smem + sizeof(ArgminSmem) + 2 * kMaxPar * sizeof(double);
    Pt<float> *pts = reinterpret_cast<Pt<float> *>(grid);
    Row<float> *rows = reinterpret_cast<Row<float> *>(grid + pts_bytes<float>(rq.n_pts));
    const PointsD P = slot_points(s);
    const MatsD Mt = slot_mats(s);
    stage_grid<float>(rq, P, Mt, pts, rows);
    if (threadIdx.x < NP) {
        s_lb[threadIdx.x] = rq.lb[threadIdx.x];
        s_ub[threadIdx.x] = rq.ub[threadIdx.x];
    }
    __syncthreads();
    const int sub = threadIdx.x % LPC;
    const int chain = threadIdx.x / LPC;
    const bool active = chain < rq.n_chains;
    const int n_mat = rq.n_mat, L = rq.chain_len, n_iters = rq.n_iters;
    const double beta = rq.beta, tmax = rq.t_max;
    auto f_of = [&](const auto *v) {
        double part = objective<MODEL, FORMULA, float, false, false, LPC>(v, pts, rows, n_mat, beta, tmax, nullptr, sub);
        part = group_sum<LPC>(part);
        return part;
    };
    double x[NP], bx[NP];
    double fx, fb, T0;
    unsigned long long nacc = 0;
    const int lev0 = s.level;
    if (s.state == SLOT_READY) {
#pragma unroll
        for (int k = 0; k < NP; ++k) x[k] = bx[k] = rq.x0[k];
        fx = f_of(x);
        fb = fx;
        T0 = rq.T0 > 0.0 ? rq.T0 : ((fx > 0.0 && fx < __builtin_inf()) ? fx : 1.0);
    } else {
        const int c = active ? chain : 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            x[k] = s.cx[c * NP + k];
            bx[k] = s.bx[c * NP + k];
        }
        fx = s.cf[c];
        fb = s.bf[c];
        nacc = s.nacc[c];
        T0 = s.T0;
    }
    const int lev1 = min(lev0 + (s.q_levels > 0 ? min(Q, s.q_levels) : Q), rq.n_levels);
    for (int lev = lev0; lev < lev1; ++lev) {
        const double h = s.sched_h[lev];
        const double Tk = T0 * s.sched_g[lev];
        const int t1 = min((lev + 1) * L, n_iters);
        if (active)
            sa_level<NP, NB, LPC, float>(chain, sub, lev * L, t1, rq.key0, rq.key1, h, Tk, s_lb, s_ub, x, fx, bx, fb,
                                         nacc, f_of);
        request_argmin<NP>(fx, chain, active, x, am, rq, 0, 0, nullptr, nullptr);
        fx = am.bf;
#pragma unroll
        for (int k = 0; k < NP; ++k) x[k] = am.bx[k];
        __syncthreads();
    }
    if (lev1 < rq.n_levels) {
        if (active && sub == 0) {
#pragma unroll
            for (int k = 0; k < NP; ++k) {
                s.cx[chain * NP + k] = x[k];
                s.bx[chain * NP + k] = bx[k];
            }
            s.cf[chain] = fx;
            s.bf[chain] = fb;
            s.nacc[chain] = nacc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s.T0 = T0;
            s.level = lev1;
            s.state = SLOT_RUNNING;
        }
        return;
    }
    // finished: best over the chains, accepted moves, polish
    request_argmin<NP>(fb, chain, active, bx, am, rq, 0, 0, nullptr, nullptr);
    unsigned long long a = (active && sub == 0) ? nacc : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
    __shared__ unsigned long long s_acc[kSlotThreads / 64];
    if ((threadIdx.x & 63) == 0) s_acc[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long tot = 0;
        for (int w = 0; w < kSlotThreads / 64; ++w) tot += s_acc[w];
        s.res_f = am.bf;
        s.res_f_pre = am.bf;
        for (int k = 0; k < NP; ++k) s.res_x[k] = am.bx[k];
        s.res_accept = tot;
        s.res_evals = 1 + (unsigned long long)rq.n_chains * (unsigned long long)rq.n_iters;
        s.level = rq.n_levels;
        s.state = rq.polish ? SLOT_POLISH : SLOT_DONE;
    }
}

// Double-precision Levenberg-Marquardt polish of a finished slot's best state
// (its own launch: one wave per slot, so that the annealing kernel keeps its
// registers for the chains).
template <int KIND>
__device__ void polish_slot_body(SlotDev &s, unsigned char *smem) {
    constexpr int MODEL = KIND == KIND_STATIC ? MODEL_STATIC : MODEL_DYN_I;
    constexpr int NP = base_npar<MODEL>();
    const ReqDesc &rq = s.rq;
    Pt<double> *pd = reinterpret_cast<Pt<double> *>(smem);
    Row<double> *rd = reinterpret_cast<Row<double> *>(smem + pts_bytes<double>(rq.n_pts));
    int32_t *prow = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(rd) + sizeof(Row<double>) * rq.n_mat);
    stage_grid<double>(rq, slot_points(s), slot_mats(s), pd, rd);
    __syncthreads();
    for (int i = 0; i < rq.n_mat; ++i)
        for (int j = rd[i].p0 + threadIdx.x; j < rd[i].p1; j += blockDim.x) prow[j] = i;
    __syncthreads();
    double xp[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) xp[k] = s.res_x[k];
    const double f_pre = s.res_f_pre;
    unsigned long long ne = 0;
    const double fp = lm_polish<MODEL, F_HAGAN, false>(xp, pd, rd, prow, rq, &ne);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (fp <= f_pre || !(f_pre < __builtin_inf())) {
            s.res_f = fp;
            for (int k = 0; k < NP; ++k) s.res_x[k] = xp[k];
        }
        s.res_evals += ne;
        s.state = SLOT_DONE;
    }
}

__global__ void __launch_bounds__(64) slot_polish_kernel(SlotDev *slots, int first) {
    SlotDev &s = slots[first + blockIdx.x];
    if (s.state != SLOT_POLISH) return;
    extern __shared__ unsigned char smem[];
    if (s.kind == KIND_STATIC)
        polish_slot_body<KIND_STATIC>(s, smem);
    else if (s.kind == KIND_DYN_I)
        polish_slot_body<KIND_DYN_I>(s, smem);
}

// One launch for every formula slot (slots [first, first + gridDim.x)): each
// workgroup runs the body of its slot's kind, so static and dynamic requests
// share the chip within one quantum.
__global__ void __launch_bounds__(kSlotThreads, 1) sa_slot_kernel(SlotDev *slots, int first, int Q) {
    SlotDev &s = slots[first + blockIdx.x];
    if (s.state != SLOT_READY && s.state != SLOT_RUNNING) return;
    extern __shared__ unsigned char smem[];
    if (s.kind == KIND_STATIC)
        sa_slot_body<KIND_STATIC>(s, Q, smem);
    else if (s.kind == KIND_DYN_I)
        sa_slot_body<KIND_DYN_I>(s, Q, smem);
}

// ---------------------------------------------------------------------------
// Monte Carlo slots (Technique II on the device): one iteration of every
// running Monte Carlo slot is three kernels: common-random-number paths for
// its (up to 64) chains, the per-chain objective, and the accept/propose
// step.  Iteration -1 evaluates f(x0) and initialises the chains.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool mc_slot_live(const SlotDev &s) {
    return s.kind == KIND_MC && (s.state == SLOT_READY || s.state == SLOT_RUNNING) && s.iter < s.sa.n_iters;
}

// Path block blockIdx.x % kMcPBlocks of Monte Carlo slot blockIdx.x / kMcPBlocks.
__global__ void __launch_bounds__(64) mc_slot_crn_kernel(SlotDev *slots) {
    SlotDev &s = slots[blockIdx.x / kMcPBlocks];
    if (!mc_slot_live(s)) return;
    extern __shared__ unsigned char smem[];
    McCrnDesc d = s.crn;
    if (s.iter < 0) d.n_chains = 1;   // f(x0) from Y[0] = x0
    crn_block<MODEL_STATIC, kCrnPaths, kCrnLdsNormals, ACC_HBM>(d, 0, blockIdx.x % kMcPBlocks, s.Y, s.msteps, s.offs,
                                                              s.K, s.part, smem);
}

// Prices and squared errors of the slot's options: block (slot, g) takes the
// options o = g, g + kMcPriceGroups, ... (four waves split the path blocks).
__global__ void __launch_bounds__(256) mc_slot_prices_kernel(SlotDev *slots) {
    SlotDev &s = slots[blockIdx.x];
    if (!mc_slot_live(s)) return;
    __shared__ double s_sum[256];
    McCrnDesc d = s.crn;
    if (s.iter < 0) d.n_chains = 1;
    for (int o = blockIdx.y; o < d.n_obs; o += kMcPriceGroups) {
        crn_price_tile(d, 0, o, s.part, s.obsrow, s.disc, s.target, s.sw, nullptr, s.e2, 64, s_sum);
        __syncthreads();
    }
}

// Objective of each chain of the slot (options added in order).
__global__ void __launch_bounds__(64) mc_slot_objective_kernel(SlotDev *slots) {
    SlotDev &s = slots[blockIdx.x];
    if (!mc_slot_live(s)) return;
    McCrnDesc d = s.crn;
    if (s.iter < 0) d.n_chains = 1;
    if (threadIdx.x < d.n_chains) s.fy[threadIdx.x] = crn_chain_objective(d, threadIdx.x, s.Y, s.e2, 64);
}

__global__ void __launch_bounds__(256) mc_slot_step_kernel(SlotDev *slots) {
    SlotDev &s = slots[blockIdx.x];
    if (!mc_slot_live(s)) return;
    __shared__ double s_f[256];
    __shared__ int s_id[256];
    const int t = s.iter;
    mc_step_body(s.sa, t, s.sched_g, s.sched_h, s.fy, s.Y, s.mcst, s.cx, s.cf, s.bx, s.bf, s_f, s_id);
    __syncthreads();
    if (threadIdx.x == 0) {
        s.iter = t + 1;
        s.state = SLOT_RUNNING;
        if (t + 1 == s.sa.n_iters) {
            mc_final_body(s.sa, s.bx, s.bf, s.mcst);
            s.res_f = s.mcst->best_f;
            s.res_f_pre = s.mcst->best_f;
            for (int k = 0; k < s.sa.n_par; ++k) s.res_x[k] = s.mcst->best_x[k];
            s.res_accept = s.mcst->n_accept;
            s.res_evals = 1 + (unsigned long long)s.sa.n_chains * (unsigned long long)s.sa.n_iters;
            s.state = SLOT_DONE;
        }
    }
}

// Status of every slot, for the host (copied back after each quantum).
__global__ void slot_status_kernel(const SlotDev *slots, int first, int n_slots, SlotStatus *st) {
    const int i = first + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= first + n_slots) return;
    const SlotDev &s = slots[i];
    SlotStatus o;
    o.state = s.state;
    o.level = s.level;
    o.iter = s.iter;
    o.pad = 0;
    o.f = s.res_f;
    o.f_pre = s.res_f_pre;
    for (int k = 0; k < kMaxPar; ++k) o.x[k] = s.res_x[k];
    o.n_accept = s.res_accept;
    o.n_evals = s.res_evals;
    st[i] = o;
}

const void *slot_prepare_kernel_ptr() { return (const void *)slot_prepare_kernel; }
const void *sa_slot_kernel_ptr() { return (const void *)sa_slot_kernel; }
const void *slot_polish_kernel_ptr() { return (const void *)slot_polish_kernel; }
const void *mc_slot_crn_kernel_ptr() { return (const void *)mc_slot_crn_kernel; }
const void *mc_slot_prices_kernel_ptr() { return (const void *)mc_slot_prices_kernel; }
const void *mc_slot_objective_kernel_ptr() { return (const void *)mc_slot_objective_kernel; }
const void *mc_slot_step_kernel_ptr() { return (const void *)mc_slot_step_kernel; }
const void *slot_status_kernel_ptr() { return (const void *)slot_status_kernel; }
size_t sa_slot_smem_bytes() {
    return sizeof(ArgminSmem) + 2 * kMaxPar * sizeof(double) + pts_bytes<float>(kSlotMaxPts) +
           sizeof(Row<float>) * kSlotMaxMat;
}
size_t slot_polish_smem_bytes() {
    return pts_bytes<double>(kSlotMaxPts) + sizeof(Row<double>) * kSlotMaxMat + sizeof(int32_t) * kSlotMaxPts;
}

}  // namespace sabr
