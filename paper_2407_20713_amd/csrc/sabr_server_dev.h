// sabr_server_dev.h -- the device-resident slot table of the serving loop.
#pragma once
#include "sabr_kernels.h"

namespace sabr {

enum SlotState : int32_t { SLOT_FREE = 0, SLOT_NEW = 1, SLOT_READY = 2, SLOT_RUNNING = 3, SLOT_DONE = 4, SLOT_POLISH = 5 };
enum SlotKind : int32_t { KIND_STATIC = 0, KIND_DYN_I = 1, KIND_MC = 2 };

constexpr int kSlotThreads = 512;   // one workgroup per formula slot
constexpr int kSlotMaxPts = 1024;
constexpr int kSlotMaxMat = 32;
constexpr int kMcPBlocks = 512;     // path blocks of one Monte Carlo slot (16384 paths: 32 a block)
constexpr int kMcPriceGroups = 32;  // option groups of the per-slot price launch
// Options of one Monte Carlo slot.  Its path blocks add their sums straight
// into HBM, so a block's LDS holds the normals and the strikes only (3.4 KB
// at this maximum, far from limiting the waves per CU): one launch with
// that LDS covers every Monte Carlo slot.
constexpr int kSlotMaxMcObs = 600;

// One slot of the serving table (device memory).  Pointers address the
// request's own region of the server's arena; grid offsets are slot-local.
struct SlotDev {
    ReqDesc rq;              // n_wg = 1; pt_off = mat_off = 0
    int32_t state, kind, level;
    int32_t q_levels;        // levels this slot advances per quantum (at most the server's Q)
    // grid: raw inputs and normalised values (slot-local CSR)
    const double *K;         // [n_pts]
    double *lfk, *lkf, *P1, *Z, *Q1, *Q2, *target, *sw;   // [n_pts]
    int32_t *row;            // [n_pts]
    double *T, *fwd, *lnf, *F1, *disc;                    // [n_mat]
    int32_t *offs;           // [n_mat + 1]
    const double *sched_g, *sched_h;                       // [n_levels]
    // annealing state, kept between quanta
    double *cx, *cf, *bx, *bf;                             // [chains * NP], [chains]
    unsigned long long *nacc;                              // [chains]
    double T0;
    // Monte Carlo objective (kind == KIND_MC)
    McCrnDesc crn;           // n_chains, n_paths, paths_per_block, grid sizes, key
    McSaDesc sa;             // model, n_par, chains, iterations, bounds, key
    McSaState *mcst;
    double *Y, *fy;          // [chains * NP], [chains]
    float *part;             // [obs][kMcPBlocks][64]
    double *e2;              // [obs][64] squared errors
    int32_t *msteps, *obsrow;  // [n_mat], [n_obs]
    int32_t iter;            // next Monte Carlo iteration (-1: initial evaluation pending)
    int32_t pad1;
    // result (state == SLOT_DONE)
    double res_f, res_f_pre;
    double res_x[kMaxPar];
    unsigned long long res_accept, res_evals;
};

// What the host reads back after each quantum.
struct SlotStatus {
    int32_t state, level, iter, pad;
    double f, f_pre;
    double x[kMaxPar];
    unsigned long long n_accept, n_evals;
};

const void *slot_prepare_kernel_ptr();
const void *sa_slot_kernel_ptr();
const void *mc_slot_crn_kernel_ptr();
const void *mc_slot_prices_kernel_ptr();
const void *mc_slot_objective_kernel_ptr();
const void *mc_slot_step_kernel_ptr();
const void *slot_status_kernel_ptr();
size_t sa_slot_smem_bytes();
size_t slot_polish_smem_bytes();
const void *slot_polish_kernel_ptr();

}  // namespace sabr
