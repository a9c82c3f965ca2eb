/*
 * fpt.h -- C ABI of the MI355X (gfx950) first-passage-time library.
 *
 * The library integrates many independent Langevin trajectories of single-field
 * inflation in the phase space (phi, pi = dphi/dN), M_pl = 1, each from
 * (phi_in, pi_in) until its first passage through phi_end, with Euler-Maruyama
 * steps, 1D noise, an importance-sampling drift bias and accumulated
 * log-weights, and reduces the first-passage times N to a weighted histogram of
 * P(deltaN), deltaN = N - N_ref.
 * Method: Jackson et al., "Stochastic inflation beyond slow roll: noise
 * modelling and importance sampling", arXiv:2410.13683:
 *   Langevin system .......................... Sec. 2.3, eq. (stochstic_eom)
 *   Euler-Maruyama step ...................... Sec. 4.1, eq. (euler_step_phi_and_pi)
 *   1D noise, biased 1D step ................. Sec. 4.1, eqs. (stochastic_eom_1D),
 *                                              (importance_sampling_1D_noise_step)
 *   bias parallel to the noise, B = A S ...... Sec. 4.1, eq. (2D_1D_noise_diussion_based_bias)
 *   weight w = exp(-sum dA) .................. Sec. 4.1, eqs. (weight), (weight_A)
 *   first-passage time, deltaN ............... Sec. 2.3 and Sec. 4.1
 *   noise table .............................. Sec. 3.2, eq. (covariance_constant_nu);
 *                                              Sec. 3.4, eq. (nu_squared_approximation)
 *   piecewise-linear potential ............... Sec. 4.2, eq. (potential_starobinsky)
 *
 * Step n of a trajectory (n = 0, 1, ...), from state (phi, pi):
 *   xi      = unit Gaussian number n of the trajectory (see "Random numbers")
 *   r       = V'(phi)/V(phi)
 *   (S, t)  = noise table at phi (S = sqrt(Xi_phiphi), t = tan theta_n)
 *   a       = bias amplitude (0, the constant A, or the learned a(phi, pi))
 *   phi'    = phi + (pi + a S) dN + S xi sqrt(dN)
 *   pi'     = pi - (3 - pi^2/2)(pi + r) dN + t (a S dN + S xi sqrt(dN))
 *   ln w   -= a xi sqrt(dN) + a^2 dN / 2            (only where S > 0)
 *   if phi' <= phi_end: N = n dN + dN (phi - phi_end)/(phi - phi')   -> done
 *   else if pi'^2 / 2 >= 1: N = (n + 1) dN, flagged "ended early"      -> done
 *   A trajectory that reaches max_steps steps without either is "censored".
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = (seed low
 * 32 bits, seed high 32 bits) and counter = (trajectory low 32 bits, n >> 2,
 * trajectory high 32 bits, instance).  Its words w0..w3 give uniforms
 * u_j = (w_j + 1/2) 2^-32 and, by Box-Muller, xi_{4m}, xi_{4m+1} =
 * rho cos(2 pi u1), rho sin(2 pi u1), rho = sqrt(-2 ln u0), and xi_{4m+2},
 * xi_{4m+3} from (u2, u3) likewise.  Trajectory indices are global
 * (traj_offset + i), so a trajectory's result does not depend on the launch
 * configuration, on how a run is split, or on which other trajectories run.
 *
 * Conventions: every function returns an int status (FPT_OK = 0, negative on
 * error) unless stated; no function aborts or throws across the ABI.  "Host"
 * pointers are ordinary CPU memory; "device" pointers are HIP device memory of
 * the current device (for example a torch tensor's data_ptr()).  A context is
 * bound to the device that is current at fpt_create and is not thread-safe:
 * use one context per concurrently used stream.
 */
#ifndef FPT_H
#define FPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------- */
enum {
    FPT_OK = 0,
    FPT_EINVAL = -1,        /* an argument is out of its documented range */
    FPT_ENOMEM = -2,        /* a device or host allocation failed */
    FPT_EHIP = -3,          /* a HIP runtime call failed */
    FPT_ESTATE = -4,        /* the call is not valid in the context's current state */
    FPT_EUNSUPPORTED = -5   /* a valid request the library does not implement */
};

/* ---- enumerations ---------------------------------------------------------- */
enum { FPT_POT_PIECEWISE_LINEAR = 0, FPT_POT_EXPONENTIAL = 1, FPT_POT_GAUSSIAN_BUMP = 2 };
enum { FPT_BIAS_NONE = 0, FPT_BIAS_CONST = 1, FPT_BIAS_MLP = 2 };
enum { FPT_FP64 = 0, FPT_FP32_STATE = 1 };
enum { FPT_BINS_LINEAR = 0, FPT_BINS_LOG = 1 };
enum { FPT_AXIS_PHI = 0, FPT_AXIS_TIME = 1 };

#define FPT_FLAG_CENSORED 0x80000000u    /* in d_steps: reached max_steps */
#define FPT_FLAG_ENDED_EARLY 0x40000000u /* in d_steps: eps_1 >= 1 before phi_end */
#define FPT_STEP_MASK 0x3fffffffu        /* in d_steps: number of steps taken */
#define FPT_MAX_STEPS 0x3fffffff
#define FPT_MAX_TABLE 4096               /* noise-table nodes (staged in LDS) */
#define FPT_MAX_BINS 1024
#define FPT_MLP_HIDDEN 64
#define FPT_MLP_NPARAM 4482              /* 2->64->64->2 network, see fpt_bias */
#define FPT_MLP_MAX_GRID 1024            /* nodes of the tabulated network */

/* ---- inputs ---------------------------------------------------------------- */

/* Potential and the start / end of the trajectories.
 *   PIECEWISE_LINEAR: eq. (potential_starobinsky), V = V0 + A_plus (phi - phi_T)
 *                     for phi >= phi_T, V0 + A_minus (phi - phi_T) for phi < phi_T.
 *   EXPONENTIAL:      V = V0 exp(A_plus (phi - phi_T)), so V'/V = A_plus everywhere
 *                     (A_minus unused).
 *   GAUSSIAN_BUMP:    eq. (potential_swagat), V = V0 phi^2/(m^2 + phi^2)
 *                     [1 + K exp(-(phi - phi_T)^2/(2 Sigma^2))], with m = bump_m,
 *                     K = bump_K, Sigma = bump_Sigma and the bump's centre phi_0 =
 *                     phi_T (A_plus, A_minus unused).  Requires m > 0, Sigma > 0,
 *                     K > -1 and phi_end > 0 (V > 0 for phi != 0).  Runs take FP64
 *                     state, 1D noise and no or a constant bias (else
 *                     FPT_EUNSUPPORTED at fpt_create), and no batches.
 * Requires finite values, phi_in > phi_end, and V > 0 on [phi_end, phi_in]. */
typedef struct {
    int32_t kind;
    double V0, phi_T, A_plus, A_minus;
    double phi_in, pi_in, phi_end;
    double bump_m, bump_K, bump_Sigma;   /* FPT_POT_GAUSSIAN_BUMP only */
} fpt_potential;

/* Noise as a function of phi (Sec. 3.2/3.4): n nodes phi_j = phi_lo + j h,
 * h = (phi_hi - phi_lo)/(n - 1).  Between nodes the values are linearly
 * interpolated; outside [phi_lo, phi_hi] the edge node applies.  n == 1 means
 * constant noise (phi_lo, phi_hi ignored).  1 <= n <= FPT_MAX_TABLE.  The host
 * arrays are copied by fpt_create.
 *   dim 0 or 1 -- 1D noise S (1, tan theta_n) xi (eq. stochastic_eom_1D):
 *     S_j = sqrt(Xi_phiphi) >= 0, tan_theta_j = Xi_phipi / Xi_phiphi.
 *   dim 2 -- 2D noise S (xi_1, xi_2) (eq. full_langevin_equation) from the node
 *     covariances Xi_pp, Xi_pq, Xi_qq (each node zero or positive definite);
 *     fpt_create takes each node's symmetric square root S and the unit
 *     principal axis e of Xi (phi component >= 0) and the kernels interpolate
 *     both.  The bias is B = a S e (the push a along e in noise space; with
 *     Xi = s s^T it is the 1D bias a s) and dA = a e.xi sqrt(dN) + a^2 |e|^2 dN/2,
 *     eq. (weight_A) for B = S (a e).  Each step takes two normals: call n >> 1
 *     of the generator, (u0, u1) for step 2m and (u2, u3) for step 2m + 1.
 *     Supported with FP64 state and no or constant bias.
 *   axis FPT_AXIS_TIME (n >= 2) -- the nodes are in the run's time instead,
 *     N_j = phi_lo + j h (phi_lo, phi_hi then hold N): step n reads the table at
 *     N = n dN.  This is the paper's own scheme (Sec. 4.1): the noise is
 *     precomputed along the classical trajectory and indexed by time, and a last
 *     node of zero switches it off after a fixed number of steps (the edge node
 *     applies beyond the table).  The FP32-state path then computes V'/V exactly
 *     every step.  1D and 2D noise; not with a learned bias (FPT_EUNSUPPORTED), nor
 *     in batches (FPT_EINVAL).  A time-indexed table of n == 1 is constant noise.
 *     fpt_noise_table_matched_time gives the Bessel-matched noise on such nodes,
 *     fpt_noise_table_bessel2d_time the 2D covariance. */
typedef struct {
    int32_t n;
    double phi_lo, phi_hi;
    const double *S;
    const double *tan_theta;
    int32_t dim;
    const double *Xi_pp, *Xi_pq, *Xi_qq;
    int32_t axis;                        /* FPT_AXIS_PHI (0) or FPT_AXIS_TIME (1) */
} fpt_noise_table;

/* Importance-sampling bias (Sec. 4.1): B_phi = a S, B_pi = tan(theta_n) a S.
 *   NONE:  a = 0 (direct sampling, w = 1).
 *   CONST: a = A (the bias amplitude).
 *   MLP:   a learned amplitude a(phi, pi) (Sec. 5 notes that the
 *          diffusion-based bias may not suffice in general and that the best
 *          bias in 2D phase space is an open question): output 0 of a 2->64->64->2
 *          network with tanh hidden layers and a linear output, whose inputs
 *          are the normalised state
 *            x0 = (phi - norm[0]) / norm[1],  x1 = (ln max(|pi|, 1e-30) - norm[2]) / norm[3].
 *          mlp_params (host, FPT_MLP_NPARAM floats, copied) is, row-major
 *          (out x in): W1[64x2] b1[64] W2[64x64] b2[64] W3[2x64] b3[2].
 *          Output 1 is not used with 1D noise.  The network is evaluated in
 *          FP64 on grid_n[0] x grid_n[1] nodes spanning x0 in [grid_range[0],
 *          grid_range[1]] and x1 in [grid_range[2], grid_range[3]] (node
 *          (i, j) at x0 = lo0 + (hi0 - lo0) i/(n0 - 1), likewise x1); a(phi, pi)
 *          is the bilinear interpolation of the node values at (x0, x1),
 *          clamped to the edge cells.  mlp_every = 0 runs this tabulated
 *          network.  mlp_every = k >= 1 makes fpt_run evaluate the network itself
 *          every k steps instead (in FP64 for FP64 state, in FP32 for FP32 state)
 *          and hold its output between evaluations: step n uses the network at the
 *          state of step k floor(n/k).  An evaluation costs about 4200 multiply-adds
 *          and 128 tanh per trajectory in FP32 state (576 tanh in FP64 state, which
 *          recomputes the first layer for every 8 units of the second); it is fastest
 *          when k divides the launch's chunk (all lanes of a wave then evaluate at
 *          the same step).
 *          The table is still built (fpt_mlp_table), and fpt_mlp_grad, whose replay
 *          uses the table, needs mlp_every = 0 (else FPT_EUNSUPPORTED).  Any
 *          deterministic function of the state is an admissible control; the
 *          weights use the same a, so the estimates stay unbiased.
 *          Requires 2 <= grid_n[k], grid_n[0] grid_n[1] <= FPT_MLP_MAX_GRID,
 *          finite norm with norm[1], norm[3] != 0, finite ranges with hi > lo. */
typedef struct {
    int32_t kind;
    double A;
    const float *mlp_params;
    double norm[4];
    int32_t mlp_every;
    int32_t grid_n[2];
    double grid_range[4];
} fpt_bias;

/* Run options.  precision: FPT_FP64 keeps (phi, pi) in FP64; FPT_FP32_STATE
 * keeps them as unevaluated float pairs updated with FP32 arithmetic (ln w,
 * the passage interpolation and the histogram stay FP64).  Histogram of
 * deltaN = N - N_ref over n_bins bins (1..FPT_MAX_BINS): LINEAR edges
 * lo + j (hi - lo)/n_bins, LOG edges lo (hi/lo)^(j/n_bins) (lo > 0); bins are
 * half-open [e_j, e_{j+1}), plus one underflow and one overflow bin.  The bin
 * of x is floor(t) with t = (x - lo) * (n_bins/(hi - lo)) (LINEAR) or
 * t = ln(x/lo) * (n_bins/ln(hi/lo)) (LOG, x <= 0 is underflow), in FP64.
 * max_steps: 1..FPT_MAX_STEPS.  instance: the fourth Philox counter word.
 * block_size (64..1024, multiple of 64), blocks_per_cu (>= 1) and chunk
 * (steps between retire/refill, multiple of 4; FP32 state steps in groups of
 * 16, 4 with mlp_every > 0, and rounds it up to a multiple of the group) select
 * the launch; 0 picks the built-in default.  They never change results. */
typedef struct {
    int32_t precision;
    int32_t bins_kind, n_bins;
    double lo, hi, N_ref;
    int64_t max_steps;
    uint32_t instance;
    int32_t block_size, blocks_per_cu, chunk;
} fpt_options;

/* Accumulated results.  The caller provides the five arrays of n_bins + 2
 * entries each (index 0 = underflow, 1..n_bins, n_bins + 1 = overflow).
 * Over trajectories that crossed phi_end: per bin count, sum w, sum w^2,
 * sum ln w, sum (ln w)^2; totals sum_w, sum_w2, sum_wN, sum_wN2.  n_traj
 * counts every trajectory run, n_steps_total every step taken.  The FP64 sums
 * are accumulated with atomics, so their last bits may vary between runs. */
typedef struct {
    uint64_t n_traj, n_censored, n_ended_early, n_steps_total;
    double sum_w, sum_w2, sum_wN, sum_wN2;
    uint64_t *count;
    double *sum_w_bin, *sum_w2_bin, *sum_lnw_bin, *sum_lnw2_bin;
} fpt_hist;

typedef struct fpt_ctx fpt_ctx;  /* opaque; owns its device table, histogram and counters */

/* ---- core API ---------------------------------------------------------------- */

/* Validate and copy the inputs, allocate the context's device memory on the
 * current device.  No kernel is launched, except that an MLP bias is
 * tabulated by a kernel on the null stream (waited for) before the return.  On success *out receives the
 * context (free it with fpt_destroy).  Errors: FPT_EINVAL (see the structs'
 * requirements; a NULL pointer; bias NULL is allowed and means NONE),
 * FPT_ENOMEM, FPT_EHIP. */
int fpt_create(const fpt_potential *pot, const fpt_noise_table *table, const fpt_bias *bias,
               const fpt_options *opts, fpt_ctx **out);

/* Run trajectories traj_offset .. traj_offset + n_traj - 1 with time step dN
 * (> 0, finite) and the 64-bit seed, asynchronously on hip_stream (a
 * hipStream_t of the context's device; NULL = the null stream).  The results
 * are added to the context's histogram.  Optional per-trajectory outputs
 * (device memory owned by the caller, n_traj entries each, entry i for
 * trajectory traj_offset + i, any of them may be NULL): d_N (N; NaN if
 * censored; the time of the end if ended early), d_lnw (ln w), d_steps (steps
 * taken | FPT_FLAG_*).  n_traj == 0 is a no-op.  The buffers must stay valid
 * until the stream reaches the end of the run.  Errors: FPT_EINVAL,
 * FPT_EHIP. */
int fpt_run(fpt_ctx *ctx, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset,
            void *hip_stream, double *d_N, double *d_lnw, uint32_t *d_steps);

/* Wait for the context's last run (fpt_run or a batch run) to finish and copy the accumulated
 * histogram to *out (host).  Only that run is waited for, through the context's own event and
 * stream, not other streams or contexts on the device; a caller that ran the context on several
 * streams orders them itself.  Errors: FPT_EINVAL (NULL arrays), FPT_EHIP. */
int fpt_histogram(fpt_ctx *ctx, fpt_hist *out);

/* Zero the accumulated histogram after the context's last run (waited for as in fpt_histogram);
 * returns when the accumulators are zero. */
int fpt_reset(fpt_ctx *ctx);

/* Wait for outstanding runs and free the context (NULL is allowed). */
void fpt_destroy(fpt_ctx *ctx);

/* Duration in milliseconds of the last fpt_run's kernel, measured with HIP
 * events recorded on the run's stream around the launch (waits for it). */
int fpt_last_kernel_ms(fpt_ctx *ctx, double *ms);

/* Static text for a status code. */
const char *fpt_strerror(int status);

/* Text describing the last error of the calling thread ("" if none). */
const char *fpt_last_error(void);

/* ---- learned bias: inference and training ------------------------------------ */

/* The context's network parameters (FPT_BIAS_MLP contexts only).  fpt_mlp_set
 * copies FPT_MLP_NPARAM floats from params (host or device memory), clears the
 * Adam moments and step count, and tabulates the network again; fpt_mlp_get
 * copies the parameters out (host or device memory) and waits for the copy.
 * Both are ordered on hip_stream: runs on other streams must be ordered after
 * it by the caller, and the source of fpt_mlp_set must stay valid until the
 * stream has reached the copy.  Errors: FPT_EINVAL (NULL, not an MLP
 * context), FPT_ESTATE (wrong current device), FPT_EHIP. */
int fpt_mlp_set(fpt_ctx *ctx, const float *params, void *hip_stream);
int fpt_mlp_get(fpt_ctx *ctx, float *params, void *hip_stream);

/* The tabulated amplitudes, node (i, j) at a_out[i grid_n[1] + j] (host array
 * of grid_n[0] grid_n[1] doubles).  Waits for the device first. */
int fpt_mlp_table(fpt_ctx *ctx, double *a_out);

/* Gradient of the tail second moment J(theta) = E[w^2 1_T], T = {trajectories
 * that crossed phi_end with deltaN = N - N_ref >= tail_lo}, at the context's
 * current parameters theta, estimated from trajectories traj_offset ..
 * traj_offset + n_traj - 1 sampled with the current control (seed, dN as in
 * fpt_run; the context's histogram is not touched):
 *   J = (1/n) sum_T w^2,
 *   dJ/dtheta = (1/n) sum_T w^2 sum_k (-xi_k sqrt(dN)) da(x_k)/dtheta,
 * the on-policy value of the replay gradient of E_old[w_old w_theta 1_T]
 * (minimising J minimises the log-weight variance on the tail under the
 * lognormal weight model of Sec. 4.1).  Tail trajectories are integrated again
 * (replayed from their counter-based random numbers) to accumulate the
 * grid-node weights G_c = (1/n) sum_T w^2 sum_k (-xi_k sqrt(dN)) beta_c(x_k),
 * which are propagated through the network at the nodes.  objective
 * FPT_MLP_OBJ_J gives dJ/dtheta; FPT_MLP_OBJ_LOG_J gives d ln J/dtheta =
 * (dJ/dtheta)/J (J divided out on the device), whose scale does not depend on
 * how rare T is (J ~ P_T^2), which suits optimisers with absolute
 * tolerances such as Adam's eps.  Outputs: d_grad
 * (device, FPT_MLP_NPARAM floats, required; all zero when no trajectory is in
 * T), d_G (device, grid_n[0] grid_n[1]
 * doubles, or NULL), J_out and n_tail_out (host, or NULL; if either is given
 * the call waits for the device).  Asynchronous on hip_stream otherwise;
 * device scratch of about 36 bytes per trajectory (at most 2^22 at a time) is
 * allocated on first use and kept.  Errors: FPT_EINVAL, FPT_ENOMEM, FPT_EHIP. */
enum { FPT_MLP_OBJ_J = 0, FPT_MLP_OBJ_LOG_J = 1 };
int fpt_mlp_grad(fpt_ctx *ctx, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset, double tail_lo,
                 int32_t objective, void *hip_stream, float *d_grad, double *d_G, double *J_out,
                 uint64_t *n_tail_out);

/* fpt_mlp_grad for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same computation, arguments and results, with
 * its per-trajectory scratch in a fixed device array of the library (about 9.4 MB per GPU the
 * library runs on, held until the process ends) instead of memory allocated on first use.  It calls
 * no hipMalloc or hipFree.  n_traj is at most FPT_MLP_GRAD_NOALLOC_MAX (else FPT_EINVAL with a
 * message; fpt_mlp_grad has no such limit).  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other threads, other contexts) race and must be ordered by the
 * caller.  Errors: as fpt_mlp_grad (FPT_ENOMEM aside), FPT_EHIP if the array's address cannot be
 * obtained. */
#define FPT_MLP_GRAD_NOALLOC_MAX 262144
int fpt_mlp_grad_noalloc(fpt_ctx *ctx, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                         double tail_lo, int32_t objective, void *hip_stream, float *d_grad, double *d_G,
                         double *J_out, uint64_t *n_tail_out);

/* One Adam step (Kingma and Ba, 2015) on the context's parameters with the
 * gradient d_grad (device, FPT_MLP_NPARAM floats): m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, theta -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * t = the context's step count + 1, computed in FP64 and stored in FP32; then
 * the network is tabulated again.  Ordered on hip_stream.  Errors: FPT_EINVAL
 * (lr <= 0, b1 or b2 outside [0, 1), eps <= 0, non-finite values), FPT_EHIP. */
int fpt_mlp_adam(fpt_ctx *ctx, const float *d_grad, double lr, double beta1, double beta2, double eps,
                 void *hip_stream);

/* ---- noise table ------------------------------------------------------------- */

/* Fill S_out[n], tan_out[n] (host arrays owned by the caller) with the noise of
 * eq. (covariance_constant_nu) -- Bunch-Davies Bessel coefficients evaluated at
 * -k eta = sigma -- with nu(phi) from eq. (nu_squared_approximation) and
 * H^2 = V(phi)/3, at the nodes phi_j = phi_lo + j (phi_hi - phi_lo)/(n - 1)
 * (n == 1: phi_lo).  The values are computed by a device kernel on the current
 * device.  Errors: FPT_EINVAL (n out of 1..FPT_MAX_TABLE, sigma <= 0,
 * V <= 0 or nu^2 <= 0 at a node), FPT_EHIP. */
int fpt_noise_table_bessel(const fpt_potential *pot, double sigma, int32_t n, double phi_lo,
                           double phi_hi, double *S_out, double *tan_out);

/* Fill Xpp_out, Xpq_out, Xqq_out (host arrays of n) with the 2D noise covariance
 * of eq. (covariance_matrix_direct): the full mode function of eq. (delta_phi_bessel)
 * with the Bunch-Davies coefficients of eq. (A_k_and_B_k) -- exact for constant nu,
 * nu(phi) from eq. (nu_squared_approximation) -- and its N-derivative at
 * -k eta = sigma, H^2 = V(phi)/3:
 *   Xi = H^2/(2 pi^2) [[|F|^2, Re(F G*)], [., |G|^2]],  F = y^(3/2)(A J_nu + B Y_nu),
 *   G = -y dF/dy,  y = sigma,
 * evaluated by the power series of J_nu and J_-nu (Y_nu = (J_nu cos nu pi -
 * J_-nu)/sin nu pi) on the device.  det Xi = (H^2 sigma^3/(4 pi^2))^2.  Errors:
 * FPT_EINVAL (n out of 1..FPT_MAX_TABLE, sigma outside (0, 2], V <= 0, nu^2 <= 0
 * or nu within 1e-3/pi of an integer at a node), FPT_EHIP. */
int fpt_noise_table_bessel2d(const fpt_potential *pot, double sigma, int32_t n, double phi_lo, double phi_hi,
                             double *Xpp_out, double *Xpq_out, double *Xqq_out);

/* Fill S_out[n], tan_out[n] and, unless NULL, fac_out[n] (host arrays owned by
 * the caller) with the Bessel-matched noise of eq. (covariance_constant_nu_bessel_matched)
 * (Sec. 3.4) at the nodes phi_j = phi_lo + j (phi_hi - phi_lo)/(n - 1):
 *   S_j = S_j^BD sqrt(fac_j),  fac_j = 4 |B_k|^2 / pi,  tan_j = nu(phi_j) - 3/2,
 * where S_j^BD is fpt_noise_table_bessel's node and B_k comes from the mode that
 * crosses the coarse-graining scale, k = sigma a H, when the classical trajectory
 * started at (phi_start, pi_start) at N = 0 passes phi_j: that mode starts at
 * k = 100 aH in the Bunch-Davies state of eq. (bunch_davies) (with the first
 * correction of the Hankel function's large-argument expansion), is evolved
 * through eq. (full_delta_phi) (RK4, FP64; the kink of the piecewise-linear
 * potential, a delta function in V'', changes d dphi/dN by
 * -(A_+ - A_-) dphi/(H^2 |pi|)) and is matched by eq. (bessel_matching) with
 * nu = nu(phi_j) of eq. (nu_squared_approximation) at -k eta = sigma.  In that
 * matching the N-derivative of (a/sqrt(-eta)) dphi is (a/sqrt(-eta))
 * (3/2 dphi + d dphi/dN), which reproduces the Bunch-Davies coefficients of
 * eq. (A_k_and_B_k) from the Bunch-Davies mode.  The matching's denominator is
 * the Bessel Wronskian, -2/pi, so B_k needs J_nu only and every nu > 0 works.  A node at or above phi_start, or
 * never reached (the trajectory is followed until phi < phi_lo, eps1 >= 1 or
 * N > 200), keeps fac = 1.  A node at phi_T takes the mode before the kink.
 * Computed by device kernels on the current device (a one-thread trajectory
 * kernel, then one thread per node; about 50 MB of device scratch for the call).
 * Errors: FPT_EINVAL (n out of 1..FPT_MAX_TABLE, sigma outside (0, 2], V <= 0 or
 * nu^2 <= 0 at a node, non-finite or eps1 >= 1 start, or a reached node whose
 * mode would start before N = 0 -- start the trajectory earlier), FPT_EHIP. */
int fpt_noise_table_matched(const fpt_potential *pot, double sigma, int32_t n, double phi_lo, double phi_hi,
                            double phi_start, double pi_start, double *S_out, double *tan_out, double *fac_out);

/* The Bessel-matched noise of fpt_noise_table_matched on nodes in time, for a
 * table of axis FPT_AXIS_TIME: node j is the time tau_j = t_lo + j (t_hi -
 * t_lo)/(n - 1) after the classical trajectory from (phi_start, pi_start) passes
 * phi_ref (normally the run's phi_in, so that the run's time n dN is tau).  The
 * node takes the trajectory's phi_j and pi_j at N_sigma = N_ref + tau_j (cubic
 * Hermite interpolation of phi between samples 1e-4 e-folds apart, linear of pi),
 * the Bunch-Davies node and nu(phi_j), and the factor 4|B_k|^2/pi of the mode
 * that crosses k = sigma a H at N_sigma.  Outputs (host, n each; fac_out and
 * phi_out may be NULL): S_out, tan_out, fac_out, phi_out = phi_j.  Errors:
 * FPT_EINVAL (sizes, sigma outside (0, 2], phi_start <= phi_ref, a trajectory
 * that does not pass phi_ref, a node before N = 0 or after the trajectory ends
 * (eps1 >= 1 or N > 200), a mode that would start before N = 0, V <= 0 or
 * nu^2 <= 0 at a node), FPT_EHIP. */
int fpt_noise_table_matched_time(const fpt_potential *pot, double sigma, int32_t n, double t_lo, double t_hi,
                                 double phi_start, double pi_start, double phi_ref, double *S_out, double *tan_out,
                                 double *fac_out, double *phi_out);

/* The 2D covariance of fpt_noise_table_bessel2d (eq. covariance_matrix_direct)
 * on nodes in time, for a 2D table of axis FPT_AXIS_TIME (Sec. 4.1: the noise
 * precomputed along the classical trajectory and read by the run's time).  Node j
 * is the time tau_j = t_lo + j (t_hi - t_lo)/(n - 1) after the classical
 * trajectory from (phi_start, pi_start) passes phi_ref, and takes the covariance
 * at the trajectory's phi there, found as in fpt_noise_table_matched_time (the
 * node at tau = 0 is phi_ref itself).  Outputs (host, n each; phi_out may be
 * NULL): Xpp_out, Xpq_out, Xqq_out, phi_out = phi_j.  Computed by device kernels
 * on the current device (about 50 MB of device scratch for the call).  Errors:
 * FPT_EINVAL (sizes, sigma outside (0, 2], phi_start <= phi_ref, a trajectory
 * that does not pass phi_ref, a node before N = 0 or after the trajectory ends,
 * V <= 0, nu^2 <= 0 or nu within 1e-3 of an integer at a node), FPT_EHIP. */
int fpt_noise_table_bessel2d_time(const fpt_potential *pot, double sigma, int32_t n, double t_lo, double t_hi,
                                  double phi_start, double pi_start, double phi_ref, double *Xpp_out,
                                  double *Xpq_out, double *Xqq_out, double *phi_out);

/* ---- batches: many problems in one persistent launch ------------------------- */

/* Several contexts (each its own potential, noise table, bias amplitude,
 * histogram, step cap and Philox instance word) integrated by one persistent
 * kernel launch.  Each instance has a trajectory cursor of its own.  Each block
 * takes a ticket naming one instance from a queue that spreads the blocks over
 * the instances in proportion to their estimated cost, stages that instance's
 * table and histogram in LDS, claims its trajectories until none is left,
 * flushes the histogram into the instance's context and takes the next ticket
 * (skipping instances with nothing left); when the tickets are used up it joins
 * any instance that still has trajectories.  Results are identical to fpt_run
 * on each context with the same seed and trajectory range.  The launch is
 * captured in a hipGraph on the first run on a (non-null) stream and replayed
 * afterwards with the new work list, seed and dN.  The contexts must share the
 * device and the precision; NONE and CONST biases may be mixed; MLP is not
 * supported here.  Per-trajectory outputs are not produced. */
typedef struct fpt_batch fpt_batch;

typedef struct {
    int32_t block_size;   /* 64..1024, multiple of 64; 0 = 1024 (or the tuned value) */
    int32_t chunk;        /* steps between retire/refill, multiple of 4 (rounded up to a multiple
                             of 16 for FP32 state); 0 = 128 */
    int32_t item_size;    /* sets the number of tickets: one per item_size trajectories in total,
                             shared among the instances by estimated cost; 0 = k x block_size with
                             k in 1..16 chosen for about 32 tickets per resident block */
    int32_t use_graph;    /* 1 = capture/replay the launch as a hipGraph (non-null streams) */
} fpt_batch_options;

/* Create a batch over ctx[0..n_inst-1] (the contexts must outlive it).
 * opts may be NULL (defaults, no graph).  Errors: FPT_EINVAL (mixed devices
 * or precisions, an MLP bias, tables/histograms too large for LDS),
 * FPT_ESTATE (wrong current device), FPT_EHIP. */
int fpt_batch_create(fpt_ctx *const *ctx, int32_t n_inst, const fpt_batch_options *opts, fpt_batch **out);

/* Run n_traj[i] trajectories of instance i (indices traj_offset ..
 * traj_offset + n_traj[i] - 1, host array of n_inst counts, zeros allowed)
 * asynchronously on hip_stream; results accumulate into each context
 * (read them with fpt_histogram).  Errors: FPT_EINVAL, FPT_ESTATE, FPT_EHIP. */
int fpt_batch_run(fpt_batch *b, const uint64_t *n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                  void *hip_stream);

/* Pick the block size and chunk for this batch: look the configuration up in
 * cache_path (text lines "key block chunk"; may be NULL), else time a probe
 * launch for each of block {256, 512, 1024} x chunk {32, 64, 128, 256} on
 * about 8192 trajectories per compute unit (spread over the instances in
 * proportion to n_traj, capped at 2^15 steps, one ticket per block_size
 * trajectories) beyond index 2^62 with private accumulators, keep the fastest,
 * measure each instance's mean steps per trajectory for the work order and
 * append the result to cache_path.  Contexts' histograms are not touched.
 * Synchronous.  Errors: FPT_EINVAL, FPT_EHIP. */
int fpt_batch_autotune(fpt_batch *b, const uint64_t *n_traj, double dN, uint64_t seed, const char *cache_path,
                       void *hip_stream);

/* The block size and chunk the batch currently uses. */
int fpt_batch_config(fpt_batch *b, int32_t *block_size, int32_t *chunk);

/* Duration in milliseconds of the last batch launch (HIP events on its stream; waits for it). */
int fpt_batch_last_ms(fpt_batch *b, double *ms);

/* Free the batch (waits for the device; NULL is allowed). */
void fpt_batch_destroy(fpt_batch *b);

/* ---- normalisation (Sec. 4.1) ----------------------------------------------- */

/* Sec. 4.1 reconstructs the distribution of the first-passage time from the weighted runs: with
 * w = exp(ln w) per trajectory (w = 1 without a bias), the estimate of P(deltaN) in a bin is the
 * bin's sum of w over n_traj times the bin width (the plain importance-sampling estimator; every
 * trajectory run counts in n_traj, also the censored and the ones that ended early).  These calls
 * work on a histogram read with fpt_histogram (host memory, the layout of fpt_hist, the bins of
 * fpt_options), run on the host and need no device. */

/* Whole-run figures of a histogram. */
typedef struct {
    double mean_w;      /* sum_w / n_traj over the trajectories that crossed phi_end: the estimate
                           of P(passage); 1 for a complete run without a bias */
    double mean_N;      /* the weighted mean passage time sum_wN / sum_w */
    double var_N;       /* the weighted variance sum_wN2 / sum_w - mean_N^2 */
    double ess;         /* effective sample size (sum_w)^2 / sum_w2 */
    double mass_under;  /* sum_w / n_traj of the underflow slot (deltaN below the first edge) */
    double mass_over;   /* sum_w / n_traj of the overflow slot (deltaN at or above the last edge) */
} fpt_moments;

/* Density of deltaN per bin: density_out[j] = sum_w_bin[j + 1] / (n_traj (e_{j+1} - e_j)) for
 * j = 0 .. n_bins - 1, with the edges e_j of fpt_options (LINEAR lo + j (hi - lo)/n_bins, LOG
 * lo (hi/lo)^(j/n_bins)).  edges_out (n_bins + 1 doubles) and m may be NULL.  bins_kind, n_bins,
 * lo and hi must be the context's.  Errors: FPT_EINVAL (NULL h, h's arrays or density_out,
 * n_bins outside 1..FPT_MAX_BINS, hi <= lo, lo <= 0 for LOG bins, n_traj == 0, a non-finite
 * sum, sum_w == 0 when m is requested). */
int fpt_density(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi, double *density_out,
                double *edges_out, fpt_moments *m);

/* A tail set T of the histogram: the slots slot .. n_bins + 1 (overflow included), i.e.
 * deltaN >= x_star.  P = sum_T w / n_traj estimates P(deltaN >= x_star); its plain standard error
 * is sqrt((sum_T w^2 / n_traj - P^2) / n_traj); ESS_T = (sum_T w)^2 / sum_T w^2, the number of
 * equally weighted samples worth as much (its relative error is about 1/sqrt(ESS_T)). */
typedef struct {
    int32_t slot;       /* first slot of T: 1 .. n_bins + 1; -1 if no slot qualifies (fpt_tail_find) */
    double x_star;      /* lower edge of T: e_{slot - 1} (hi for the overflow slot) */
    double P;
    double P_err;
    double P_err_lognormal; /* the per-slot lognormal one-sigma half-widths (hi - lo)/2 of
                               fpt_lognormal_bins over the slots of T, added in quadrature (slots
                               with fewer than 2 samples contribute nothing; 0 without sum_lnw arrays) */
    double ess;
    uint64_t count;     /* trajectories in T */
} fpt_tail;

/* The tail set from a given first slot (1 .. n_bins + 1).  Errors: FPT_EINVAL (as fpt_density, or
 * slot out of range). */
int fpt_tail_at(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi, int32_t slot,
                fpt_tail *out);

/* The tail set at a target probability: the lowest slot whose tail mass sum_{slots >= j} w / n_traj
 * is positive and at most p_target (the depth the estimate reaches).  out->slot = -1 and zeros
 * when none is.  Errors: FPT_EINVAL (as fpt_density, or p_target not positive and finite). */
int fpt_tail_find(const fpt_hist *h, int32_t bins_kind, int32_t n_bins, double lo, double hi, double p_target,
                  fpt_tail *out);

/* ---- error bars (Sec. 4.1) -------------------------------------------------- */

/* Histogram slots throughout: n_slots = n_bins + 2 (underflow, the bins, overflow),
 * the layout of fpt_hist.  "Mass" is sum_w / n_traj of a slot; divide by the bin
 * width for the density.  All arrays are host memory owned by the caller; these
 * calls run on the host and need no device. */

/* Direct sampling: the paper resamples independent runs.  Delete-one jackknife over
 * n_blocks >= 2 blocks of trajectories (for example consecutive fpt_run calls, each
 * read with fpt_histogram and cleared with fpt_reset).  n_traj[b] is block b's
 * trajectory count; sum_w is row-major [n_blocks][n_slots].  p_out is the mass of
 * all blocks together.  err_out is sqrt((B - 1)/B sum_b (p_(b) - mean p_(b))^2),
 * where p_(b) = (sum sum_w - sum_w[b]) / (sum n - n_b).  Errors: FPT_EINVAL (sizes,
 * NULL, a block with no trajectories, non-finite sums). */
int fpt_jackknife(int32_t n_slots, int32_t n_blocks, const uint64_t *n_traj, const double *sum_w, double *p_out,
                  double *err_out);

/* Importance sampling: the paper takes the error of a slot from the error of the
 * mean of a lognormal distribution.  Within slot j the n_j = count[j] values of
 * ln w are taken as normal, with mean mu = sum_lnw/n_j and variance
 * s^2 = (sum_lnw2 - n_j mu^2)/(n_j - 1).  Outputs:
 *   p_out  = (n_j/n_traj) exp(mu + s^2/2);
 *   lo_out, hi_out = p_out exp(-+se), the one-sigma interval of ln(mass), with
 *            se^2 = s^2/n_j + s^4/(2 (n_j - 1))  (Cox's, for ln of the mean weight)
 *                 + (1 - n_j/n_traj)/n_j         (the count's binomial fluctuation).
 * With constant weights the interval is the binomial one.  All three are NaN where
 * n_j < 2.  The inputs are fpt_hist's count, sum_lnw_bin and sum_lnw2_bin.
 * Errors: FPT_EINVAL (sizes, NULL, n_traj == 0). */
int fpt_lognormal_bins(int32_t n_slots, uint64_t n_traj, const uint64_t *count, const double *sum_lnw,
                       const double *sum_lnw2, double *p_out, double *lo_out, double *hi_out);

/* Several bias amplitudes: the inverse-variance weighted mean per slot over n_runs
 * runs, p and err row-major [n_runs][n_slots].  In each slot, a run with a
 * non-finite value or error, or an error <= 0, is left out.  p_out = sum (p/err^2)
 * / sum (1/err^2) and err_out = 1/sqrt(sum (1/err^2)); both are NaN where no run is
 * left.  Errors: FPT_EINVAL (sizes, NULL). */
int fpt_merge_bins(int32_t n_slots, int32_t n_runs, const double *p, const double *err, double *p_out,
                   double *err_out);

#ifdef __cplusplus
}
#endif

#endif /* FPT_H */
