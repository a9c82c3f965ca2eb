// internal.hpp -- structures shared by the library's translation units (not
// part of the public ABI; see include/fpt.h for that).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

#include "potential.hpp"

namespace fpt {

enum : int { kPotPiecewiseLinear = 0, kPotExponential = 1, kPotGaussianBump = 2 };
enum : int { kBiasNone = 0, kBiasConst = 1, kBiasMlp = 2 };
// kernel-side bias variant (not in the ABI): the learned control's network evaluated exactly every
// mlp_every steps instead of read from its table
constexpr int kBiasMlpExact = 3;
enum : int { kBinsLinear = 0, kBinsLog = 1 };

constexpr uint32_t kFlagCensored = 0x80000000u;
constexpr uint32_t kFlagEndedEarly = 0x40000000u;
constexpr uint32_t kStepMask = 0x3fffffffu;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = 4482;
// parameter offsets (row-major, out x in): W1[64x2] b1[64] W2[64x64] b2[64] W3[2x64] b3[2]
constexpr int kOffW1 = 0, kOffB1 = 128, kOffW2 = 192, kOffB2 = 4288, kOffW3 = 4352, kOffB3 = 4480;
constexpr int kMlpMaxGrid = 1024;    // nodes of the tabulated network

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

// One first-passage problem as the kernels see it: potential, start and end,
// noise table, bias, step cap, Philox instance word and histogram target.
struct Inst {
    int32_t pot_kind;
    double V0, phi_T, A_plus, A_minus;
    double phi_in, pi_in, phi_end;
    // Gaussian bump (pot_kind 2): m^2, K, Sigma; the centre phi_0 is phi_T
    double bump_m2, bump_K, bump_Sigma;
    // noise table: n_tab nodes from phi_lo with spacing 1/inv_h, in phi (tab_axis 0) or in the
    // run's time N = n dN (tab_axis 1: phi_lo and inv_h then refer to N)
    int32_t n_tab, tab_axis;
    double phi_lo, inv_h;
    const double2 *tab64;            // node j: (S_j, tan_j)                                  (device)
    const float4 *tab32;             // node j: (S_j, S_j+1 - S_j, tan_j, tan_j+1 - tan_j) in FP32
    // FP32 V'/V per table interval j: (r_j, r_j+1 - r_j) of the interval's own branch of the
    // potential, or NaN where V'/V must be computed exactly (see fpt_api.hip)
    const float2 *rtab32;
    // over the FP32 records whose V'/V interval is a number (the smooth ones): the largest |S_j|,
    // |S_j+1 - S_j|, |tan_j|, |tan_j+1 - tan_j|, |V'/V_j| and |V'/V_j+1 - V'/V_j|, which bound what
    // a group evaluating one record for all its steps can read (all 0 without a smooth record)
    float rec_S, rec_dS, rec_t, rec_dt, rec_r, rec_dr;
    int32_t all_S_pos;               // every node has S > 0 (the ln w update needs no test)
    // 2D noise (noise_dim == 2): node j is (S_pp, S_pq), (S_qq, e_phi), (e_pi, 0) -- the symmetric
    // square root of the node covariance and its unit principal axis
    int32_t noise_dim;
    const double2 *tab64_2d;
    // the same in FP32 for FP32 state, three float4 per node: (S_pp, slope, S_pq, slope),
    // (S_qq, slope, e_phi, slope), (e_pi, slope, V'/V interval value, slope) -- the interval as in rtab32
    const float4 *tab32_2d;
    int32_t bias_kind;
    double A;
    // learned amplitude tabulated on g_n0 x g_n1 nodes of the normalised inputs;
    // grid coordinates u0 = phi g_k0 + g_off0, u1 = ln max(|pi|, 1e-30) g_k1 + g_off1
    int32_t g_n0, g_n1;
    double g_k0, g_off0, g_k1, g_off1;
    const double2 *grid64;           // cell c = i0 (n1 - 1) + i1: [2c] = (a00, a10), [2c+1] = (a01, a11)
    const float4 *grid32;            // cell c: (a00, a10, a01, a11) in FP32
    // the network itself (fpt_run with mlp_every >= 1): its FP32 parameters and the normalised
    // inputs x0 = phi m_k0 + m_off0, x1 = ln max(|pi|, 1e-30) m_k1 + m_off1
    int32_t mlp_every;
    const float *mlp_params;
    double m_k0, m_off0, m_k1, m_off1;
    uint32_t instance;               // fourth Philox counter word
    uint32_t max_steps;
    HistSpec hist;
    void *acc;                       // global accumulators (acc_bytes(hist.n_bins))
};

// Per-run values shared by every instance of a launch.
struct RunArgs {
    double dN, sqrt_dN;
    uint32_t key0, key1;             // Philox key = seed
    int32_t chunk;                   // steps between retire/refill (multiple of 4; whole step groups are run)
};

// One launch of the single-problem Euler-Maruyama kernel.
struct EmParams {
    Inst inst;
    RunArgs run;
    uint64_t traj_offset, n_traj;
    double *d_N, *d_lnw;             // optional per-trajectory outputs (device, caller-owned)
    uint32_t *d_steps;
    unsigned long long *cursor;      // work-queue head (relative trajectory index)
};

// A slice of one instance's trajectories, processed by one block of the batch kernel.
// One entry of a batch's work list: instance inst and its whole trajectory range
// [begin, begin + count) of the run (tickets and the per-instance entries alike).
struct WorkItem {
    uint32_t inst;
    uint32_t pad;
    uint64_t begin, count;
};

// Device-resident parameters of a batch launch (read by the kernel, so a
// captured graph can be replayed with new values).
struct BatchRun {
    RunArgs run;
    uint64_t n_items;      // tickets at the start of the work list
    uint64_t n_inst;       // per-instance entries after them
};

// One entry of the list of trajectories whose gradient contribution is replayed.
struct TailEntry {
    uint64_t traj;                   // global trajectory index
    double ww;                       // w_old w_theta of the path (w^2 on-policy)
};

// One launch of the replay kernel: the trajectories of `tail`, integrated again
// with the instance's tabulated control, scatter their per-step gradient factors
// onto the grid nodes `d_G` (n0 n1 doubles, accumulated with atomics).
struct ReplayParams {
    Inst inst;
    RunArgs run;
    const TailEntry *tail;
    const unsigned long long *n_tail;  // device count of entries
    double *d_G;
    unsigned long long *cursor;
    unsigned long long *mismatch;      // replays that did not end with a passage
};

// Euler-Maruyama kernels (fpt_em.hip).
__host__ __device__ inline int grid_cells(const Inst &I) { return I.bias_kind == kBiasMlp ? (I.g_n0 - 1) * (I.g_n1 - 1) : 0; }
size_t em_lds_bytes(int n_bins, int n_tab, int precision, int n_cells, bool mlp_exact = false);
size_t replay_lds_bytes(int n_tab, int precision, int n_cells, int n_nodes);
// tab_mode: 0 a single node, 1 nodes in phi, 2 nodes in time (tab_mode(inst)); pot_kind selects
// the Gaussian-bump variant (FP64, bias none or constant only).
const void *em_kernel_ptr(int precision, int bias_kind, int tab_mode, bool all_pos, int pot_kind = 0);
hipError_t em_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream,
                     bool mlp_exact = false);
const void *replay_kernel_ptr(int precision, bool all_pos);
size_t em2d_lds_bytes(int n_bins, int n_tab, int precision);
const void *em2d_kernel_ptr(int precision, int bias_kind, bool all_pos, bool time_axis);
hipError_t em2d_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream);
hipError_t replay_launch(const ReplayParams &p, int precision, int grid, int block, hipStream_t stream);
const void *batch_kernel_ptr(int precision, int bias_kind, bool all_pos);
// cursors: [0] the ticket cursor, [1 + i] instance i's trajectory cursor (zeroed before each launch)
hipError_t batch_launch(int precision, int bias_kind, bool all_pos, const Inst *insts, const WorkItem *items,
                        const BatchRun *run, unsigned long long *cursors, int max_bins, int max_tab, int grid,
                        int block, hipStream_t stream);
hipError_t zero_words(unsigned long long *ptr, size_t n, hipStream_t stream);

// Learned-control kernels (fpt_mlp.hip).  params: 4482 FP32 values,
// W1[64x2] b1 W2[64x64] b2 W3[2x64] b3; the network is evaluated in FP64.
struct GridSpec {
    int32_t n0, n1;
    double lo0, hi0, lo1, hi1;       // ranges of the normalised inputs covered by the nodes
};
hipError_t mlp_tabulate(const float *params, const GridSpec &g, double *node_a, double2 *grid64, float4 *grid32,
                        hipStream_t stream);
hipError_t mlp_tail_compact(const double *d_N, const double *d_lnw, const uint32_t *d_steps, uint64_t n,
                            uint64_t traj_offset, double N_ref, double tail_lo, TailEntry *tail,
                            unsigned long long *n_tail, unsigned long long *n_tail_total, double *J_sum,
                            hipStream_t stream);
// grad[4482] (FP32) = sum_c G_c / den d a(x_c)/d theta over the grid nodes, with
// den = *d_den when d_den is given (a device value; den = 0 gives a zero gradient),
// else n_scale; work: 4 n0 n1 64 doubles of scratch.
hipError_t mlp_backprop(const float *params, const GridSpec &g, const double *G, double n_scale,
                        const double *d_den, double *work, float *grad, hipStream_t stream);
hipError_t mlp_scale_copy(const double *src, double scale, double *dst, size_t n, hipStream_t stream);
hipError_t mlp_adam(float *params, float *m, float *v, const float *grad, int n, double lr, double beta1,
                    double beta2, double eps, double bc1, double bc2, hipStream_t stream);

// Bessel-matched noise table (fpt_table.hip).  Scratch: kMatchCap trajectory samples
// (N, phi, pi) then n + 1 ints; matched_scratch_bytes(n) bytes.  d_status collects
// 1 (V <= 0 or nu^2 <= 0 at a node), 2 (a node reached before its mode can start),
// 4 (non-finite or zero B_k).
constexpr int kMatchCap = (1 << 21) + 16;
size_t matched_scratch_bytes(int n);
hipError_t matched_table_launch(const PotParams &pot, double sigma, int n, double phi_lo, double h_node,
                                double phi_start, double pi_start, void *scratch, double *d_S, double *d_tan,
                                double *d_fac, int *d_status, hipStream_t stream);
// Time nodes N_ref + t_lo + j h after the trajectory passes phi_ref; the trajectory is followed
// until N_ref + N_after.  Scratch: matched_time_scratch_bytes().  d_status as above plus 16 (no
// passage of phi_ref, or a node outside the followed trajectory).
size_t matched_time_scratch_bytes();
hipError_t matched_time_launch(const PotParams &pot, double sigma, int n, double t_lo, double h, double phi_start,
                               double pi_start, double phi_ref, double N_after, void *scratch, double *d_S,
                               double *d_tan, double *d_fac, double *d_phi, int *d_status, hipStream_t stream);
// The 2D Bunch-Davies covariance on the same time nodes (scratch as above; d_status 1 or 16).
hipError_t bessel2d_time_launch(const PotParams &pot, double sigma, int n, double t_lo, double h, double phi_start,
                                double pi_start, double phi_ref, double N_after, void *scratch, double *d_Xpp,
                                double *d_Xpq, double *d_Xqq, double *d_phi, int *d_status, hipStream_t stream);

// Sets the message fpt_last_error returns and returns code (defined in fpt_api.hip).
int report_error(int code, const char *msg);

// Node j of a table grid, lo + j h, rounded as two separate operations (no fused multiply-add), so
// that a node meant to sit on a point (a kink, a reference time) lands on the same double as in a
// plain IEEE evaluation.
__device__ inline double grid_node(double lo, int j, double h)
{
#pragma clang fp contract(off)
    return lo + (double)j * h;
}

// The table mode of the kernels: a single node, nodes in phi, or nodes in time.
__host__ __device__ inline int tab_mode(const Inst &I) { return I.n_tab > 1 ? (I.tab_axis ? 2 : 1) : 0; }

}  // namespace fpt
