// sabr_kernels.h -- launch descriptors and kernel handles shared by the host
// runtime and the kernel translation units.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "sabr_dev.h"

namespace sabr {

// Monte Carlo pricing of one parameter set (lane = path).
struct McDesc {
    int32_t model, n_mat, n_obs, m_max;
    int64_t n_paths;
    double dt, f0, beta;
    double x[kMaxPar];
    uint32_t key0, key1;
    int32_t anti, pad;   // antithetic path pairs
};

// Common-random-number Monte Carlo of many parameter sets (lane = set).
struct McCrnDesc {
    int32_t n_mat, n_obs, m_max, n_pblocks;
    int64_t n_chains, n_paths, paths_per_block;
    int32_t np_stride, beta_free;
    double dt, f0, beta;
    uint32_t key0, key1;
    int32_t model, anti;   // anti: antithetic path pairs
    double t_max;
};

// Annealing with the Monte Carlo objective (one request).
struct McSaDesc {
    int32_t model, n_par, n_chains, n_iters, chain_len;
    uint32_t key0, key1;
    double T0, t_max;
    double lb[kMaxPar], ub[kMaxPar], x0[kMaxPar];
};
struct McSaState {
    double T0;
    unsigned long long n_accept;
    double best_f;
    double best_x[kMaxPar];
};

// At-the-money start point of one grid (one wave).
struct AtmDesc {
    int32_t n_mat, n_par, beta_free, pad;
    double beta;
    double lb[kMaxPar], ub[kMaxPar];
};

// Cliquet on the Monte Carlo paths of one parameter set (lane = path).
struct CliqDesc {
    int32_t model, n_reset, m_max, anti;   // anti: antithetic path pairs
    int64_t n_paths;
    double dt, f0, beta;
    double x[kMaxPar];
    double local_floor, local_cap, global_floor, global_cap;
    uint32_t key0, key1;
};

// Kernel handles (the kernels are templates instantiated in the .hip files).
const void *atm_seed_kernel_ptr();
const void *prepare_points_kernel_ptr();
const void *prepare_mats_kernel_ptr();
const void *objective_kernel_ptr(int model, int formula, bool fp32, bool bfree);
const void *sa_kernel_ptr(int model, int formula, bool fp32, bool bfree, int lpc);
bool wide_lanes_supported(int model, bool fp32);   // 4, 8 or 16 lanes per chain
const void *polish_kernel_ptr(int model, int formula, bool bfree);
size_t grid_smem_bytes(bool fp32, int n_pts, int n_mat);
size_t sa_smem_fixed_bytes();

const void *mc_price_kernel_ptr(bool fp32);
const void *mc_price_finalize_ptr();
const void *mc_grid_kernel_ptr();
const void *mc_cliquet_kernel_ptr(bool fp32);
size_t mc_cliquet_smem_bytes(bool fp32, int m_max);
const void *mc_crn_kernel_ptr(int model, int variant);
const void *mc_crn_direct_kernel_ptr(int model);
int mc_crn_direct_paths();   // paths per block of the direct kernel
const void *mc_crn_prices_ptr();
const void *mc_crn_objective_ptr();
const void *mc_sa_step_ptr();
const void *mc_sa_final_ptr();
size_t mc_price_smem_bytes(bool fp32, int m_max, int n_obs);
size_t mc_crn_smem_bytes(int n_obs, bool direct = false);

}  // namespace sabr
