// internal.hpp -- structures shared by the library's translation units (not
// part of the public ABI; see include/fpt.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace fpt {

enum : int { kPotPiecewiseLinear = 0, kPotExponential = 1 };
enum : int { kBiasNone = 0, kBiasConst = 1, kBiasMlp = 2 };
enum : int { kBinsLinear = 0, kBinsLog = 1 };

constexpr uint32_t kFlagCensored = 0x80000000u;
constexpr uint32_t kFlagEndedEarly = 0x40000000u;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 4482;

// Histogram of deltaN = N - N_ref.  scale = n_bins/(hi - lo) for linear bins,
// n_bins/ln(hi/lo) for log bins.
struct HistSpec {
    int32_t bins_kind, n_bins;
    double lo, scale, N_ref;
};

// Accumulators, identical in LDS (per block) and in global memory (per
// context).  Word layout, nb = n_bins + 2:
//   uint64  count[nb]
//   uint64  ucnt[4]      n_censored, n_ended_early, n_steps_total, (unused)
//   double  sum_w[nb], sum_w2[nb], sum_lnw[nb], sum_lnw2[nb]
//   double  dtot[4]      sum_w, sum_w2, sum_wN, sum_wN2
__host__ __device__ inline size_t acc_words(int n_bins) { return (size_t)(n_bins + 2) * 5 + 8; }
__host__ __device__ inline size_t acc_bytes(int n_bins) { return acc_words(n_bins) * 8; }

// Everything one launch of the Euler-Maruyama kernel needs.
struct EmParams {
    // potential (eq. potential_starobinsky; exponential companion)
    int32_t pot_kind;
    double V0, phi_T, A_plus, A_minus;
    double phi_in, pi_in, phi_end;
    // phi-indexed noise table: n_tab nodes from phi_lo with spacing 1/inv_h
    int32_t n_tab;
    double phi_lo, inv_h;
    const double2 *tab64;            // node j: (S_j, tan_j)                        (device)
    const float4 *tab32;             // node j: (S_j, S_j+1 - S_j, tan_j, tan_j+1 - tan_j) in FP32
    int32_t all_S_pos;               // every node has S > 0 (the ln w update needs no test)
    // importance-sampling bias
    int32_t bias_kind;
    double A;
    const float *mlp;                // device, kMlpParams floats
    double norm[4];
    int32_t mlp_every;
    // run
    double dN, sqrt_dN;
    uint32_t key0, key1, instance;
    uint64_t traj_offset, n_traj;
    uint32_t max_steps;
    int32_t chunk;
    HistSpec hist;
    // outputs
    double *d_N, *d_lnw;
    uint32_t *d_steps;
    unsigned long long *cursor;      // work-queue head (relative trajectory index)
    void *acc;                       // global accumulators (acc_bytes(n_bins))
};

// Euler-Maruyama kernels (fpt_em.hip).
size_t em_lds_bytes(const EmParams &p, int precision);
const void *em_kernel_ptr(const EmParams &p, int precision);
hipError_t em_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream);
hipError_t zero_words(unsigned long long *ptr, size_t n, hipStream_t stream);

}  // namespace fpt
