/*
 * fpt_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the stochastic-deltaN
 * first-passage method of Jackson, Assadullahi, Gow, Koyama, Vennin, Wands,
 * "Stochastic inflation beyond slow roll: noise modelling and importance
 * sampling" (arXiv:2410.13683).  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this file.  It shares no code, header,
 * constant or helper with the GPU library, and it does not include or link
 * anything from it.
 *
 * What it follows (sections / equations of the paper):
 *   - Langevin system in (phi, pi = dphi/dN), M_pl = 1:        Sec. 2.3, eq. (stochstic_eom)
 *   - Euler-Maruyama step:                                      Sec. 4.1, eq. (euler_step_phi_and_pi)
 *   - 1D noise S_phiphi (1, tan theta_n):                       Sec. 4.1, eq. (stochastic_eom_1D)
 *   - importance-sampled 1D step (sign of the drift restored):  Sec. 4.1, eq. (importance_sampling_1D_noise_step)
 *   - bias parallel to the noise, diffusion-based amplitude:    Sec. 4.1, constraint below eq. (importance_sampling_1D_noise_step)
 *                                                               and eq. (2D_1D_noise_diussion_based_bias)
 *   - weight w = exp(-sum dA), dA of the Mazonka form:          Sec. 4.1, eqs. (weight), (weight_A)
 *   - first-passage time N = n dN, deltaN = N - <N>:            Sec. 4.1 and Sec. 2.3
 *   - piecewise-linear potential:                               Sec. 4.2, eq. (potential_starobinsky)
 *   - Gaussian-bump potential:                                  Sec. 4.3, eq. (potential_swagat)
 *   - constant-nu noise with Bunch-Davies coefficients:         Sec. 3.2, eq. (covariance_constant_nu)
 *   - nu^2 as a function of phi only after the transition:      Sec. 3.4, eq. (nu_squared_approximation)
 *   - 2D noise from the full Bunch-Davies mode, general weight:  Sec. 3.3, eq. (covariance_matrix_direct);
 *                                                               Sec. 2.3, eq. (full_langevin_equation)
 *   - Bessel-matched noise from the mode equation:              Sec. 2.1, eqs. (full_delta_phi), (bunch_davies);
 *                                                               Sec. 3.4, eqs. (bessel_matching),
 *                                                               (covariance_constant_nu_bessel_matched)
 *   - noise precomputed along the classical trajectory and read
 *     by the run's time, switched off after a fixed time:       Sec. 4.1
 *
 * Readings where the paper is silent or garbled (the design notes list each):
 *   - the drift in the biased pi step carries the same minus sign as in the
 *     unbiased step;
 *   - the bias is parallel to the noise vector: B_pi = tan(theta_n) B_phi with
 *     B_phi = A S_phiphi (the printed constraint has the two sides swapped);
 *   - dA in 1D is eq. (weight_A) restricted to the noise direction:
 *     dA = (B_phi dN / 2 + S_phiphi xi sqrt(dN)) B_phi / S_phiphi^2, and 0 where S = 0;
 *   - absorption when phi <= phi_end; N is interpolated linearly in phi over
 *     the crossing step; eps_1 = pi^2/2 >= 1 before phi_end only raises a flag;
 *   - the noise is a function of phi (linear interpolation of a uniform table,
 *     clamped to the edge nodes), H^2 = V/3 inside the table; a table may
 *     instead have its nodes in the run's time, read at N = n dN;
 *   - random numbers: Philox4x32-10 keyed by the 64-bit seed, counter
 *     (step>>2, trajectory lo, trajectory hi, instance); the four 32-bit words
 *     give four uniforms u = (w + 1/2) 2^-32 and two Box-Muller pairs.
 *
 * Parity status: every function below is pinned by a CPU test under tests/
 * (test_oracle_*.py); the learned-bias replay gradient is pinned by central
 * finite differences of its own objective.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int orc_threads(int n_threads);

#define ORC_POT_PIECEWISE_LINEAR 0
#define ORC_POT_EXPONENTIAL 1
#define ORC_POT_GAUSSIAN_BUMP 2

#define ORC_BIAS_NONE 0
#define ORC_BIAS_CONST 1
#define ORC_BIAS_MLP 2

#define ORC_FLAG_CENSORED 0x80000000u
#define ORC_FLAG_ENDED_EARLY 0x40000000u
#define ORC_STEP_MASK 0x3fffffffu

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplications,     */
/* the key advanced by the Weyl constants between rounds.                     */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k[0] += W0;
        k[1] += W1;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* The unit Gaussian xi of step n of trajectory `traj` (global index) of
 * instance `instance`.  Call m = n >> 2 of the generator, on the counter
 * (traj lo, m, traj hi, instance) and the key (seed lo, seed hi), yields four words;
 * u_j = (w_j + 1/2) / 2^32 lies strictly inside (0, 1).  Box-Muller (1958):
 * (u0, u1) -> rho cos(2 pi u1), rho sin(2 pi u1) with rho = sqrt(-2 ln u0),
 * and (u2, u3) likewise; xi_n is entry n & 3 of these four. */
static void orc_four_normals(uint64_t seed, uint32_t instance, uint64_t traj, uint64_t m, double z[4])
{
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)m, (uint32_t)(traj >> 32), instance};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    double u[4];
    for (int j = 0; j < 4; ++j) u[j] = ((double)w[j] + 0.5) / 4294967296.0;
    const double two_pi = 2.0 * M_PI;
    double rho01 = sqrt(-2.0 * log(u[0]));
    double rho23 = sqrt(-2.0 * log(u[2]));
    z[0] = rho01 * cos(two_pi * u[1]);
    z[1] = rho01 * sin(two_pi * u[1]);
    z[2] = rho23 * cos(two_pi * u[3]);
    z[3] = rho23 * sin(two_pi * u[3]);
}

/* xi_n for n = n0 .. n0+count-1 (exported for the tests). */
void orc_normals(uint64_t seed, uint32_t instance, uint64_t traj, uint64_t n0, uint64_t count, double *z_out)
{
    for (uint64_t i = 0; i < count; ++i) {
        uint64_t n = n0 + i;
        double z[4];
        orc_four_normals(seed, instance, traj, n >> 2, z);
        z_out[i] = z[n & 3];
    }
}

/* Uniforms u_j of call m (exported for the Box-Muller invariance tests). */
void orc_uniforms(uint64_t seed, uint32_t instance, uint64_t traj, uint64_t m, double u_out[4])
{
    uint32_t ctr[4] = {(uint32_t)traj, (uint32_t)m, (uint32_t)(traj >> 32), instance};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    for (int j = 0; j < 4; ++j) u_out[j] = ((double)w[j] + 0.5) / 4294967296.0;
}

/* ------------------------------------------------------------------------- */
/* Potentials.  pot = {V0, phi_T, A_plus, A_minus, m, K, Sigma}.              */
/*   piecewise linear, eq. (potential_starobinsky):                           */
/*       V = V0 + A_+ (phi - phi_T) for phi >= phi_T, V0 + A_- (phi - phi_T)  */
/*       otherwise (phi == phi_T takes the A_+ branch);                       */
/*   exponential: V = V0 exp(A_+ (phi - phi_T)), for which V'/V = A_+ exactly */
/*       and pi = -A_+ is an exact fixed point of the drift;                  */
/*   Gaussian bump, eq. (potential_swagat):                                   */
/*       V = V0 u(phi) (1 + g(phi)),  u = phi^2/(m^2 + phi^2),                */
/*       g = K exp(-x^2/2),  x = (phi - phi_0)/Sigma,  phi_0 = phi_T.         */
/* ------------------------------------------------------------------------- */
/* u, g and their first two derivatives for the Gaussian bump. */
static void orc_bump_parts(const double pot[7], double phi, double u[3], double g[3])
{
    const double m2 = pot[4] * pot[4], K = pot[5], Sig = pot[6];
    const double q = m2 + phi * phi;
    u[0] = phi * phi / q;
    u[1] = 2.0 * m2 * phi / (q * q);
    u[2] = 2.0 * m2 * (m2 - 3.0 * phi * phi) / (q * q * q);
    const double x = (phi - pot[1]) / Sig;
    g[0] = K * exp(-0.5 * x * x);
    g[1] = -x / Sig * g[0];
    g[2] = (x * x - 1.0) / (Sig * Sig) * g[0];
}

double orc_V(int kind, const double pot[7], double phi)
{
    const double V0 = pot[0], phi_T = pot[1], Ap = pot[2], Am = pot[3];
    if (kind == ORC_POT_EXPONENTIAL) return V0 * exp(Ap * (phi - phi_T));
    if (kind == ORC_POT_GAUSSIAN_BUMP) {
        double u[3], g[3];
        orc_bump_parts(pot, phi, u, g);
        return V0 * u[0] * (1.0 + g[0]);
    }
    if (phi >= phi_T) return V0 + Ap * (phi - phi_T);
    return V0 + Am * (phi - phi_T);
}

double orc_dV(int kind, const double pot[7], double phi)
{
    const double phi_T = pot[1], Ap = pot[2], Am = pot[3];
    if (kind == ORC_POT_EXPONENTIAL) return Ap * orc_V(kind, pot, phi);
    if (kind == ORC_POT_GAUSSIAN_BUMP) {
        double u[3], g[3];
        orc_bump_parts(pot, phi, u, g);
        return pot[0] * (u[1] * (1.0 + g[0]) + u[0] * g[1]);
    }
    return (phi >= phi_T) ? Ap : Am;
}

double orc_d2V(int kind, const double pot[7], double phi)
{
    const double Ap = pot[2];
    if (kind == ORC_POT_EXPONENTIAL) return Ap * Ap * orc_V(kind, pot, phi);
    if (kind == ORC_POT_GAUSSIAN_BUMP) {
        double u[3], g[3];
        orc_bump_parts(pot, phi, u, g);
        return pot[0] * (u[2] * (1.0 + g[0]) + 2.0 * u[1] * g[1] + u[0] * g[2]);
    }
    (void)phi;
    return 0.0; /* linear on each side of phi_T */
}

/* ------------------------------------------------------------------------- */
/* Noise table of eq. (covariance_constant_nu) with nu(phi) from              */
/* eq. (nu_squared_approximation):                                            */
/*   nu^2 = 9/4 - 3 [V''/V - (V'/V)^2],  H^2 = V/3,                           */
/*   Xi_phiphi = H^2/(4 pi^2) [Gamma(nu)/Gamma(3/2)]^2 (sigma/2)^(3 - 2 nu),  */
/*   Xi_phipi  = (nu - 3/2) Xi_phiphi,                                        */
/*   S_phiphi = sqrt(Xi_phiphi),  tan theta_n = Xi_phipi / Xi_phiphi.         */
/* Nodes phi_j = phi_lo + j h, h = (phi_hi - phi_lo)/(n - 1); n == 1 gives a  */
/* single node at phi_lo.  Returns 0, or -1 on invalid input.                 */
/* ------------------------------------------------------------------------- */
int orc_noise_table_bessel(int kind, const double pot[7], double sigma, int n,
                           double phi_lo, double phi_hi, double *S_out, double *tan_out)
{
    if (n < 1 || !(sigma > 0.0)) return -1;
    if (n > 1 && !(phi_hi > phi_lo)) return -1;
    double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    for (int j = 0; j < n; ++j) {
        double phi = phi_lo + (double)j * h;
        double V = orc_V(kind, pot, phi);
        if (!(V > 0.0)) return -1;
        double dVV = orc_dV(kind, pot, phi) / V;
        double d2VV = orc_d2V(kind, pot, phi) / V;
        double nu2 = 9.0 / 4.0 - 3.0 * (d2VV - dVV * dVV);
        if (!(nu2 > 0.0)) return -1;
        double nu = sqrt(nu2);
        double H2 = V / 3.0;
        double g = tgamma(nu) / tgamma(1.5);
        double Xi_pp = H2 / (4.0 * M_PI * M_PI) * g * g * pow(sigma / 2.0, 3.0 - 2.0 * nu);
        double Xi_ppi = (nu - 1.5) * Xi_pp;
        S_out[j] = sqrt(Xi_pp);
        tan_out[j] = Xi_ppi / Xi_pp;
    }
    return 0;
}

/* Linear interpolation of the table at phi, clamped to the edge nodes. */
static void orc_table_lookup(int n_tab, double phi_lo, double phi_hi, const double *S_tab,
                             const double *t_tab, double phi, double *S, double *t)
{
    if (n_tab == 1) { *S = S_tab[0]; *t = t_tab[0]; return; }
    double h = (phi_hi - phi_lo) / (double)(n_tab - 1);
    double x = (phi - phi_lo) / h;
    double jf = floor(x);
    if (jf < 0.0) jf = 0.0;
    if (jf > (double)(n_tab - 2)) jf = (double)(n_tab - 2);
    int j = (int)jf;
    double f = x - jf;
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    *S = S_tab[j] + f * (S_tab[j + 1] - S_tab[j]);
    *t = t_tab[j] + f * (t_tab[j + 1] - t_tab[j]);
}

/* ------------------------------------------------------------------------- */
/* Learned bias amplitude: a 2 -> 64 -> 64 -> 2 network with tanh hidden      */
/* layers and a linear output, evaluated in FP64 from FP32 parameters.        */
/* Layout (4482 floats, row-major, out x in): W1[64x2] b1[64] W2[64x64]       */
/* b2[64] W3[2x64] b3[2].  Inputs x0 = (phi - c0)/s0,                         */
/* x1 = (ln max(|pi|, 1e-30) - c1)/s1 with norm = {c0, s0, c1, s1}.            */
/* Output 0 is the amplitude a(phi, pi); output 1 would bias a second noise   */
/* direction and is unused with 1D noise.                                     */
/* ------------------------------------------------------------------------- */
#define MLP_H 64
#define MLP_NPARAM 4482

static void orc_mlp_inputs(const double norm[4], double phi, double pi_, double x[2])
{
    double ap = fabs(pi_);
    if (ap < 1e-30) ap = 1e-30;
    x[0] = (phi - norm[0]) / norm[1];
    x[1] = (log(ap) - norm[2]) / norm[3];
}

/* Forward pass; also returns the hidden activations when h1/h2 are non-NULL. */
static double orc_mlp_forward(const float *p, const double x[2], double *h1_out, double *h2_out)
{
    const float *W1 = p, *b1 = p + 128, *W2 = p + 192, *b2 = p + 4288, *W3 = p + 4352, *b3 = p + 4480;
    double h1[MLP_H], h2[MLP_H];
    for (int j = 0; j < MLP_H; ++j) {
        double s = (double)b1[j];
        for (int i = 0; i < 2; ++i) s += (double)W1[j * 2 + i] * x[i];
        h1[j] = tanh(s);
    }
    for (int j = 0; j < MLP_H; ++j) {
        double s = (double)b2[j];
        for (int i = 0; i < MLP_H; ++i) s += (double)W2[j * MLP_H + i] * h1[i];
        h2[j] = tanh(s);
    }
    double out0 = (double)b3[0];
    for (int i = 0; i < MLP_H; ++i) out0 += (double)W3[i] * h2[i];
    (void)W3; /* row 1 of W3 and b3[1] feed output 1, unused for 1D noise */
    if (h1_out) memcpy(h1_out, h1, sizeof h1);
    if (h2_out) memcpy(h2_out, h2, sizeof h2);
    return out0;
}

double orc_mlp_eval(const float *params, const double norm[4], double phi, double pi_)
{
    double x[2];
    orc_mlp_inputs(norm, phi, pi_, x);
    return orc_mlp_forward(params, x, NULL, NULL);
}

/* d a / d params at (phi, pi): plain back-propagation through the network,
 * accumulated with weight `scale` into grad[4482] (FP64). */
static void orc_mlp_backward(const float *p, const double x[2], double scale, double *grad)
{
    const float *W2 = p + 192, *W3 = p + 4352;
    double h1[MLP_H], h2[MLP_H];
    orc_mlp_forward(p, x, h1, h2);
    double *gW1 = grad, *gb1 = grad + 128, *gW2 = grad + 192, *gb2 = grad + 4288, *gW3 = grad + 4352, *gb3 = grad + 4480;
    /* out0 = b3[0] + sum_i W3[0,i] h2[i] */
    gb3[0] += scale;
    double d2[MLP_H];
    for (int i = 0; i < MLP_H; ++i) {
        gW3[i] += scale * h2[i];
        d2[i] = scale * (double)W3[i] * (1.0 - h2[i] * h2[i]);
    }
    double d1[MLP_H];
    for (int i = 0; i < MLP_H; ++i) d1[i] = 0.0;
    for (int j = 0; j < MLP_H; ++j) {
        gb2[j] += d2[j];
        for (int i = 0; i < MLP_H; ++i) {
            gW2[j * MLP_H + i] += d2[j] * h1[i];
            d1[i] += d2[j] * (double)W2[j * MLP_H + i];
        }
    }
    for (int i = 0; i < MLP_H; ++i) {
        double g = d1[i] * (1.0 - h1[i] * h1[i]);
        gb1[i] += g;
        gW1[i * 2 + 0] += g * x[0];
        gW1[i * 2 + 1] += g * x[1];
    }
}

/* ------------------------------------------------------------------------- */
/* Tabulated learned amplitude: the network evaluated on a uniform grid of the  */
/* normalised inputs (x0, x1) with n0 x n1 nodes over [lo0, hi0] x [lo1, hi1],  */
/* stored row-major a[i n1 + j]; between nodes bilinear interpolation, outside  */
/* the grid the edge nodes.  Any deterministic function of the state is an      */
/* admissible control for importance sampling, and the weights use the same     */
/* function, so sampling with the tabulated network stays unbiased.             */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n0, n1;
    double lo0, hi0, lo1, hi1;
} orc_grid;

static double orc_grid_x(const orc_grid *g, int axis, int k)
{
    const int n = axis ? g->n1 : g->n0;
    const double lo = axis ? g->lo1 : g->lo0, hi = axis ? g->hi1 : g->hi0;
    return lo + (hi - lo) * (double)k / (double)(n - 1);
}

int orc_mlp_tabulate(const float *params, int n0, int n1, double lo0, double hi0, double lo1, double hi1,
                     double *a_out)
{
    if (n0 < 2 || n1 < 2 || !(hi0 > lo0) || !(hi1 > lo1)) return -1;
    orc_grid g = {n0, n1, lo0, hi0, lo1, hi1};
    for (int i = 0; i < n0; ++i)
        for (int j = 0; j < n1; ++j) {
            double x[2] = {orc_grid_x(&g, 0, i), orc_grid_x(&g, 1, j)};
            a_out[i * n1 + j] = orc_mlp_forward(params, x, NULL, NULL);
        }
    return 0;
}

/* Bilinear value at (x0, x1); the four corner indices and weights are returned. */
static double orc_grid_eval(const orc_grid *g, const double *a, double x0, double x1, int idx[4], double beta[4])
{
    double u0 = (x0 - g->lo0) / (g->hi0 - g->lo0) * (double)(g->n0 - 1);
    double u1 = (x1 - g->lo1) / (g->hi1 - g->lo1) * (double)(g->n1 - 1);
    double i0 = floor(u0), i1 = floor(u1);
    if (i0 < 0.0) i0 = 0.0;
    if (i0 > (double)(g->n0 - 2)) i0 = (double)(g->n0 - 2);
    if (i1 < 0.0) i1 = 0.0;
    if (i1 > (double)(g->n1 - 2)) i1 = (double)(g->n1 - 2);
    double f0 = u0 - i0, f1 = u1 - i1;
    if (f0 < 0.0) f0 = 0.0;
    if (f0 > 1.0) f0 = 1.0;
    if (f1 < 0.0) f1 = 0.0;
    if (f1 > 1.0) f1 = 1.0;
    const int k = (int)i0 * g->n1 + (int)i1;
    idx[0] = k; idx[1] = k + g->n1; idx[2] = k + 1; idx[3] = k + g->n1 + 1;
    beta[0] = (1.0 - f0) * (1.0 - f1);
    beta[1] = f0 * (1.0 - f1);
    beta[2] = (1.0 - f0) * f1;
    beta[3] = f0 * f1;
    return beta[0] * a[idx[0]] + beta[1] * a[idx[1]] + beta[2] * a[idx[2]] + beta[3] * a[idx[3]];
}

/* ------------------------------------------------------------------------- */
/* One trajectory, Sec. 4.1.  Writes N, ln w and the step count with flags.   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int kind;
    double pot[7];
    int n_tab;
    double phi_lo, phi_hi;
    const double *S_tab, *t_tab;
    int tab_axis;             /* 0: nodes in phi; 1: nodes in the run's time N = n dN (phi_lo, phi_hi hold N) */
    double phi_in, pi_in, phi_end;
    int bias_kind;
    double A_bias;
    const float *mlp;
    double norm[4];
    int mlp_every;            /* >= 1: the network every k steps; 0: the tabulated network */
    orc_grid grid;
    const double *grid_a;     /* tabulated amplitude (mlp_every == 0) */
    double dN;
    uint64_t seed;
    uint32_t instance;
    int64_t max_steps;
} orc_problem;

/* phi2_out (may be NULL): phi before and after the last step taken (both the current phi for a */
/* censored trajectory), what a reader needs to tell a floating-point near-tie at phi_end and a */
/* short last step apart from a real disagreement.                                               */
static void orc_trajectory(const orc_problem *P, uint64_t traj, double *N_out, double *lnw_out, uint32_t *steps_out,
                           double *phi2_out)
{
    const double dN = P->dN;
    const double sqrt_dN = sqrt(dN);
    double phi = P->phi_in, pi_ = P->pi_in, lnw = 0.0;
    int64_t n = 0;
    double zbuf[4];
    uint64_t zcall = UINT64_MAX;
    double A_held = 0.0;
    for (;;) {
        if (n >= P->max_steps) {
            *N_out = NAN;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n | ORC_FLAG_CENSORED;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi; }
            return;
        }
        /* xi^(i) */
        uint64_t call = (uint64_t)n >> 2;
        if (call != zcall) { orc_four_normals(P->seed, P->instance, traj, call, zbuf); zcall = call; }
        double xi = zbuf[n & 3];
        /* drift vector D = (pi, -(3 - pi^2/2)(pi + V'/V)), eq. (stochstic_eom) */
        double V = orc_V(P->kind, P->pot, phi);
        double dV = orc_dV(P->kind, P->pot, phi);
        double D_phi = pi_;
        double D_pi = -(3.0 - pi_ * pi_ / 2.0) * (pi_ + dV / V);
        /* 1D noise amplitude and direction at the local field value (or at the run's time) */
        double S, tan_theta;
        orc_table_lookup(P->n_tab, P->phi_lo, P->phi_hi, P->S_tab, P->t_tab, P->tab_axis ? (double)n * dN : phi,
                         &S, &tan_theta);
        /* bias amplitude A (constant or learned) and bias vector parallel to the noise */
        double A = 0.0;
        if (P->bias_kind == ORC_BIAS_CONST) {
            A = P->A_bias;
        } else if (P->bias_kind == ORC_BIAS_MLP) {
            if (P->mlp_every > 0) {
                if (n % P->mlp_every == 0) A_held = orc_mlp_eval(P->mlp, P->norm, phi, pi_);
                A = A_held;
            } else {
                double x[2];
                int idx[4];
                double beta[4];
                orc_mlp_inputs(P->norm, phi, pi_, x);
                A = orc_grid_eval(&P->grid, P->grid_a, x[0], x[1], idx, beta);
            }
        }
        double B_phi = A * S;
        double B_pi = tan_theta * B_phi;
        /* biased Euler-Maruyama step, eq. (importance_sampling_1D_noise_step) */
        double phi_next = phi + D_phi * dN + B_phi * dN + S * xi * sqrt_dN;
        double pi_next = pi_ + D_pi * dN + B_pi * dN + tan_theta * S * xi * sqrt_dN;
        /* dA of eq. (weight_A) along the single noise direction */
        if (S > 0.0) {
            double dA = (B_phi / 2.0 * dN + S * xi * sqrt_dN) * B_phi / (S * S);
            lnw -= dA;
        }
        n += 1;
        if (phi_next <= P->phi_end) {
            /* linear interpolation of the passage inside step n */
            double frac = (phi - P->phi_end) / (phi - phi_next);
            *N_out = (double)(n - 1) * dN + dN * frac;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi_next; }
            return;
        }
        if (pi_next * pi_next / 2.0 >= 1.0) {
            /* eps_1 >= 1: inflation ended before phi_end */
            *N_out = (double)n * dN;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n | ORC_FLAG_ENDED_EARLY;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi_next; }
            return;
        }
        phi = phi_next;
        pi_ = pi_next;
    }
}

/* Run n_traj trajectories with global indices traj_offset .. traj_offset+n_traj-1.
 * Returns 0, or -1 on invalid input.  n_threads <= 0 uses the OpenMP default. */
int orc_run(int kind, const double pot[7],
            int n_tab, double phi_lo, double phi_hi, const double *S_tab, const double *t_tab, int tab_axis,
            double phi_in, double pi_in, double phi_end,
            int bias_kind, double A_bias, const float *mlp_params, const double *mlp_norm,
            int mlp_every, const int grid_n[2], const double grid_range[4],
            double dN, uint64_t seed, uint32_t instance, uint64_t traj_offset, uint64_t n_traj,
            int64_t max_steps, double *N_out, double *lnw_out, uint32_t *steps_out, double *phi2_out,
            int n_threads)
{
    if (n_tab < 1 || !(dN > 0.0) || max_steps < 1 || max_steps > (int64_t)ORC_STEP_MASK) return -1;
    if (!(phi_in > phi_end)) return -1;
    if (bias_kind == ORC_BIAS_MLP && (!mlp_params || !mlp_norm || mlp_every < 0)) return -1;
    if (tab_axis && bias_kind == ORC_BIAS_MLP) return -1;
    orc_problem P;
    memset(&P, 0, sizeof P);
    double *grid_a = NULL;
    if (bias_kind == ORC_BIAS_MLP && mlp_every == 0) {
        orc_grid g = {grid_n[0], grid_n[1], grid_range[0], grid_range[1], grid_range[2], grid_range[3]};
        grid_a = (double *)malloc(sizeof(double) * (size_t)(g.n0 > 1 ? g.n0 : 1) * (size_t)(g.n1 > 1 ? g.n1 : 1));
        if (!grid_a || orc_mlp_tabulate(mlp_params, g.n0, g.n1, g.lo0, g.hi0, g.lo1, g.hi1, grid_a) != 0) {
            free(grid_a);
            return -1;
        }
        P.grid = g;
        P.grid_a = grid_a;
    }
    P.mlp_every = mlp_every;
    P.kind = kind;
    memcpy(P.pot, pot, sizeof P.pot);
    P.n_tab = n_tab; P.phi_lo = phi_lo; P.phi_hi = phi_hi; P.S_tab = S_tab; P.t_tab = t_tab;
    P.tab_axis = tab_axis ? 1 : 0;
    P.phi_in = phi_in; P.pi_in = pi_in; P.phi_end = phi_end;
    P.bias_kind = bias_kind; P.A_bias = A_bias; P.mlp = mlp_params;
    if (mlp_norm) memcpy(P.norm, mlp_norm, sizeof P.norm);
    P.dN = dN; P.seed = seed; P.instance = instance; P.max_steps = max_steps;
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    int64_t nt = (int64_t)n_traj;
#pragma omp parallel for num_threads(n_thr) schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i)
        orc_trajectory(&P, traj_offset + (uint64_t)i, &N_out[i], &lnw_out[i], &steps_out[i],
                       phi2_out ? &phi2_out[2 * i] : NULL);
    free(grid_a);
    return 0;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of one parallel region: n_threads if positive, else the OpenMP default.  A per-region */
/* count leaves the process-wide default alone.                                                   */
static int orc_threads(int n_threads)
{
    return n_threads > 0 ? n_threads : orc_max_threads();
}

/* ------------------------------------------------------------------------- */
/* Replay gradient of the learned-bias objective.                             */
/*                                                                            */
/* Paths are drawn once under the sampling amplitude a_old (the network at    */
/* the parameters that generated them).  With e_k = a_old(x_k) dN + xi_k      */
/* sqrt(dN) the noise-space increment of step k, the log-weight of the same   */
/* path under a candidate amplitude a_theta is                                */
/*     ln w_theta = sum_k ( -a_theta(x_k) e_k + a_theta(x_k)^2 dN / 2 ),      */
/* which is eq. (weight_A) with the increment written in the unbiased noise.  */
/* The objective is the second moment of the estimator on the tail set T:     */
/*     J(theta) = (1/n) sum_{paths in T} w_old w_theta,                       */
/* with gradient (1/n) sum_T w_old w_theta sum_k (-e_k + a_theta dN) grad a.  */
/* Replaying at theta = theta_old gives w_old w_theta = w^2.                  */
/* Only trajectories whose deltaN = N - N_ref lies in [tail_lo, +inf) count.  */
/* grad_out has 4482 doubles; J_out receives J(theta).                        */
/* ------------------------------------------------------------------------- */
int orc_mlp_replay_grad(int kind, const double pot[7],
                        int n_tab, double phi_lo, double phi_hi, const double *S_tab, const double *t_tab,
                        double phi_in, double pi_in, double phi_end,
                        const float *theta_old, const float *theta, const double *mlp_norm,
                        double dN, uint64_t seed, uint32_t instance, uint64_t traj_offset, uint64_t n_traj,
                        int64_t max_steps, double N_ref, double tail_lo,
                        double *grad_out, double *J_out, int n_threads)
{
    if (n_tab < 1 || !(dN > 0.0) || max_steps < 1) return -1;
    orc_problem P;
    memset(&P, 0, sizeof P);
    P.kind = kind;
    memcpy(P.pot, pot, sizeof P.pot);
    P.n_tab = n_tab; P.phi_lo = phi_lo; P.phi_hi = phi_hi; P.S_tab = S_tab; P.t_tab = t_tab;
    P.phi_in = phi_in; P.pi_in = pi_in; P.phi_end = phi_end;
    P.bias_kind = ORC_BIAS_MLP; P.mlp = theta_old; P.mlp_every = 1;
    memcpy(P.norm, mlp_norm, sizeof P.norm);
    P.dN = dN; P.seed = seed; P.instance = instance; P.max_steps = max_steps;
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    const double sqrt_dN = sqrt(dN);
    int64_t nt = (int64_t)n_traj;
    double J = 0.0;
    for (int k = 0; k < MLP_NPARAM; ++k) grad_out[k] = 0.0;
#pragma omp parallel num_threads(n_thr)
    {
        double *g_local = (double *)calloc(MLP_NPARAM, sizeof(double));
        double *g_path = (double *)calloc(MLP_NPARAM, sizeof(double));
        double J_local = 0.0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < nt; ++i) {
            uint64_t traj = traj_offset + (uint64_t)i;
            double N, lnw_old;
            uint32_t steps;
            orc_trajectory(&P, traj, &N, &lnw_old, &steps, NULL);
            if (steps & (ORC_FLAG_CENSORED | ORC_FLAG_ENDED_EARLY)) continue;
            if (!(N - N_ref >= tail_lo)) continue;
            /* replay the same path: states and noise are those drawn under theta_old */
            double phi = phi_in, pi_ = pi_in, lnw_new = 0.0;
            memset(g_path, 0, MLP_NPARAM * sizeof(double));
            uint32_t n_steps = steps & ORC_STEP_MASK;
            double zbuf[4];
            uint64_t zcall = UINT64_MAX;
            for (uint32_t n = 0; n < n_steps; ++n) {
                uint64_t call = (uint64_t)n >> 2;
                if (call != zcall) { orc_four_normals(seed, instance, traj, call, zbuf); zcall = call; }
                double xi = zbuf[n & 3];
                double V = orc_V(kind, pot, phi);
                double dV = orc_dV(kind, pot, phi);
                double S, tan_theta;
                orc_table_lookup(n_tab, phi_lo, phi_hi, S_tab, t_tab, phi, &S, &tan_theta);
                double x[2];
                orc_mlp_inputs(mlp_norm, phi, pi_, x);
                double a_old = orc_mlp_forward(theta_old, x, NULL, NULL);
                if (S > 0.0) {
                    double a_new = orc_mlp_forward(theta, x, NULL, NULL);
                    double e = a_old * dN + xi * sqrt_dN;
                    lnw_new += -a_new * e + a_new * a_new * dN / 2.0;
                    orc_mlp_backward(theta, x, -e + a_new * dN, g_path);
                }
                double B_phi = a_old * S;
                double B_pi = tan_theta * B_phi;
                double D_pi = -(3.0 - pi_ * pi_ / 2.0) * (pi_ + dV / V);
                double phi_next = phi + pi_ * dN + B_phi * dN + S * xi * sqrt_dN;
                double pi_next = pi_ + D_pi * dN + B_pi * dN + tan_theta * S * xi * sqrt_dN;
                phi = phi_next;
                pi_ = pi_next;
            }
            double ww = exp(lnw_old + lnw_new);
            J_local += ww;
            for (int k = 0; k < MLP_NPARAM; ++k) g_local[k] += ww * g_path[k];
        }
#pragma omp critical
        {
            J += J_local;
            for (int k = 0; k < MLP_NPARAM; ++k) grad_out[k] += g_local[k];
        }
        free(g_local);
        free(g_path);
    }
    for (int k = 0; k < MLP_NPARAM; ++k) grad_out[k] /= (double)n_traj;
    *J_out = J / (double)n_traj;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Replay gradient with the tabulated control.  Paths are drawn with the grid  */
/* of theta_old; a candidate theta changes the grid values, so the amplitude   */
/* at step k is a_theta,k = sum_c beta_c(x_k) net_theta(x_c) over the four     */
/* corners c of the cell holding x_k, and                                      */
/*   ln w_theta = sum_k ( -a_theta,k e_k + a_theta,k^2 dN / 2 ),               */
/*   e_k = a_old,k dN + xi_k sqrt(dN)      (steps with S > 0),                 */
/*   J(theta) = (1/n) sum_{paths in T} w_old w_theta,                          */
/*   grad J = (1/n) sum_T w_old w_theta sum_k (-e_k + a_theta,k dN)            */
/*                 sum_c beta_c(x_k) grad net_theta(x_c).                      */
/* The grid-node weights G_c are accumulated over paths first and then         */
/* propagated through the network once per node.                               */
/* ------------------------------------------------------------------------- */
int orc_grid_replay_grad(int kind, const double pot[7],
                         int n_tab, double phi_lo, double phi_hi, const double *S_tab, const double *t_tab,
                         double phi_in, double pi_in, double phi_end,
                         const float *theta_old, const float *theta, const double *mlp_norm,
                         const int grid_n[2], const double grid_range[4],
                         double dN, uint64_t seed, uint32_t instance, uint64_t traj_offset, uint64_t n_traj,
                         int64_t max_steps, double N_ref, double tail_lo,
                         double *grad_out, double *J_out, double *G_out, int n_threads)
{
    if (n_tab < 1 || !(dN > 0.0) || max_steps < 1) return -1;
    orc_grid g = {grid_n[0], grid_n[1], grid_range[0], grid_range[1], grid_range[2], grid_range[3]};
    const size_t ng = (size_t)g.n0 * (size_t)g.n1;
    double *a_old = (double *)malloc(sizeof(double) * ng);
    double *a_new = (double *)malloc(sizeof(double) * ng);
    double *G = (double *)calloc(ng, sizeof(double));
    if (!a_old || !a_new || !G || orc_mlp_tabulate(theta_old, g.n0, g.n1, g.lo0, g.hi0, g.lo1, g.hi1, a_old) ||
        orc_mlp_tabulate(theta, g.n0, g.n1, g.lo0, g.hi0, g.lo1, g.hi1, a_new)) {
        free(a_old); free(a_new); free(G);
        return -1;
    }
    orc_problem P;
    memset(&P, 0, sizeof P);
    P.kind = kind;
    memcpy(P.pot, pot, sizeof P.pot);
    P.n_tab = n_tab; P.phi_lo = phi_lo; P.phi_hi = phi_hi; P.S_tab = S_tab; P.t_tab = t_tab;
    P.phi_in = phi_in; P.pi_in = pi_in; P.phi_end = phi_end;
    P.bias_kind = ORC_BIAS_MLP; P.mlp = theta_old; P.mlp_every = 0; P.grid = g; P.grid_a = a_old;
    memcpy(P.norm, mlp_norm, sizeof P.norm);
    P.dN = dN; P.seed = seed; P.instance = instance; P.max_steps = max_steps;
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    const double sqrt_dN = sqrt(dN);
    const int64_t nt = (int64_t)n_traj;
    double J = 0.0;
#pragma omp parallel num_threads(n_thr)
    {
        double *G_local = (double *)calloc(ng, sizeof(double));
        double J_local = 0.0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t i = 0; i < nt; ++i) {
            const uint64_t traj = traj_offset + (uint64_t)i;
            double N, lnw_old;
            uint32_t steps;
            orc_trajectory(&P, traj, &N, &lnw_old, &steps, NULL);
            if (steps & (ORC_FLAG_CENSORED | ORC_FLAG_ENDED_EARLY)) continue;
            if (!(N - N_ref >= tail_lo)) continue;
            const uint32_t n_steps = steps & ORC_STEP_MASK;
            double lnw_new = 0.0, ww = 0.0;
            for (int pass = 0; pass < 2; ++pass) {
                /* pass 0: ln w_theta of the path; pass 1: its node weights, scaled by w_old w_theta */
                double phi = phi_in, pi_ = pi_in;
                double zbuf[4];
                uint64_t zcall = UINT64_MAX;
                for (uint32_t n = 0; n < n_steps; ++n) {
                    const uint64_t call = (uint64_t)n >> 2;
                    if (call != zcall) { orc_four_normals(seed, instance, traj, call, zbuf); zcall = call; }
                    const double xi = zbuf[n & 3];
                    const double V = orc_V(kind, pot, phi), dV = orc_dV(kind, pot, phi);
                    double S, tan_theta;
                    orc_table_lookup(n_tab, phi_lo, phi_hi, S_tab, t_tab, phi, &S, &tan_theta);
                    double x[2], beta[4];
                    int idx[4];
                    orc_mlp_inputs(mlp_norm, phi, pi_, x);
                    const double a_o = orc_grid_eval(&g, a_old, x[0], x[1], idx, beta);
                    if (S > 0.0) {
                        const double a_n = beta[0] * a_new[idx[0]] + beta[1] * a_new[idx[1]] +
                                           beta[2] * a_new[idx[2]] + beta[3] * a_new[idx[3]];
                        const double e = a_o * dN + xi * sqrt_dN;
                        if (pass == 0) {
                            lnw_new += -a_n * e + a_n * a_n * dN / 2.0;
                        } else {
                            const double c = ww * (-e + a_n * dN);
                            for (int q = 0; q < 4; ++q) G_local[idx[q]] += c * beta[q];
                        }
                    }
                    const double B_phi = a_o * S, B_pi = tan_theta * B_phi;
                    const double D_pi = -(3.0 - pi_ * pi_ / 2.0) * (pi_ + dV / V);
                    const double phi_next = phi + pi_ * dN + B_phi * dN + S * xi * sqrt_dN;
                    const double pi_next = pi_ + D_pi * dN + B_pi * dN + tan_theta * S * xi * sqrt_dN;
                    phi = phi_next;
                    pi_ = pi_next;
                }
                if (pass == 0) {
                    ww = exp(lnw_old + lnw_new);
                    J_local += ww;
                }
            }
        }
#pragma omp critical
        {
            J += J_local;
            for (size_t k = 0; k < ng; ++k) G[k] += G_local[k];
        }
        free(G_local);
    }
    for (int k = 0; k < MLP_NPARAM; ++k) grad_out[k] = 0.0;
    for (int i = 0; i < g.n0; ++i)
        for (int j = 0; j < g.n1; ++j) {
            const size_t k = (size_t)i * g.n1 + j;
            G[k] /= (double)n_traj;
            if (G[k] == 0.0) continue;
            double x[2] = {orc_grid_x(&g, 0, i), orc_grid_x(&g, 1, j)};
            orc_mlp_backward(theta, x, G[k], grad_out);
        }
    if (G_out) memcpy(G_out, G, sizeof(double) * ng);
    *J_out = J / (double)n_traj;
    free(a_old); free(a_new); free(G);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Adam (Kingma and Ba, "Adam: a method for stochastic optimization", 2015),   */
/* the textbook update: step t of                                              */
/*   m <- b1 m + (1 - b1) g,   v <- b2 v + (1 - b2) g^2,                       */
/*   theta <- theta - lr mhat / (sqrt(vhat) + eps),                           */
/*   mhat = m / (1 - b1^t),    vhat = v / (1 - b2^t),                          */
/* in FP64, with theta, m and v stored in FP32 between steps.                  */
/* ------------------------------------------------------------------------- */
void orc_adam_step(float *theta, float *m, float *v, const float *grad, int n, int t, double lr, double b1,
                   double b2, double eps)
{
    const double bc1 = 1.0 - pow(b1, (double)t);
    const double bc2 = 1.0 - pow(b2, (double)t);
    for (int i = 0; i < n; ++i) {
        const double g = (double)grad[i];
        const double mi = b1 * (double)m[i] + (1.0 - b1) * g;
        const double vi = b2 * (double)v[i] + (1.0 - b2) * g * g;
        m[i] = (float)mi;
        v[i] = (float)vi;
        const double mhat = mi / bc1;
        const double vhat = vi / bc2;
        theta[i] = (float)((double)theta[i] - lr * mhat / (sqrt(vhat) + eps));
    }
}

/* ========================================================================= */
/* Two-dimensional noise.                                                    */
/* ========================================================================= */

/* Noise covariance of eq. (covariance_matrix_direct): the full mode function */
/* of eq. (delta_phi_bessel) with the Bunch-Davies coefficients of            */
/* eq. (A_k_and_B_k) -- the exact mode for constant nu -- and its N-derivative */
/* at -k eta = sigma.  With y = -k eta, sqrt(-eta)/a = H (y/k)^(3/2) and        */
/* d/dN = -y d/dy:                                                             */
/*   delta phi_k = H k^(-3/2) F(y),  F = y^(3/2) [A J_nu(y) + B Y_nu(y)],       */
/*   delta pi_k  = H k^(-3/2) (-y F'(y)),                                      */
/*   Xi = k^3/(2 pi^2) [[|dphi|^2, Re(dphi dpi*)], [., |dpi|^2]]               */
/*      = H^2/(2 pi^2) [[|F|^2, Re(F conj(-y F'))], [., |y F'|^2]].             */
/* Y_nu = (J_nu cos(nu pi) - J_-nu)/sin(nu pi) and the power series            */
/* J_mu(y) = sum_m (-1)^m (y/2)^(2m + mu) / (m! Gamma(m + mu + 1)) give        */
/*   F = sum_{mu = nu, -nu} alpha_mu sum_m c_m(mu) y^(2m + mu + 3/2),           */
/*   -y F' = -sum alpha_mu sum_m (2m + mu + 3/2) c_m(mu) y^(2m + mu + 3/2),     */
/* alpha_nu = A + B cot(nu pi), alpha_-nu = -B / sin(nu pi),                   */
/* c_m(mu) = (-1)^m / (m! Gamma(m + mu + 1) 2^(2m + mu)).  The m = 0 terms are */
/* the homogeneous growing (mu = -nu) and decaying (mu = nu) modes of          */
/* eq. (bessel_matched_homogeneous).  30 terms per series: for sigma <= 2 the  */
/* remainder is below 1e-40 of the leading term.  nu and H^2 = V/3 as for the  */
/* 1D table.                                                                    */
/* ------------------------------------------------------------------------- */
int orc_noise_table_bessel2d(int kind, const double pot[7], double sigma, int n, double phi_lo, double phi_hi,
                             double *Xpp_out, double *Xpq_out, double *Xqq_out)
{
    if (n < 1 || !(sigma > 0.0) || sigma > 2.0) return -1;
    if (n > 1 && !(phi_hi > phi_lo)) return -1;
    const double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    for (int j = 0; j < n; ++j) {
        const double phi = phi_lo + (double)j * h;
        const double V = orc_V(kind, pot, phi);
        if (!(V > 0.0)) return -1;
        const double dVV = orc_dV(kind, pot, phi) / V;
        const double d2VV = orc_d2V(kind, pot, phi) / V;
        const double nu2 = 9.0 / 4.0 - 3.0 * (d2VV - dVV * dVV);
        if (!(nu2 > 0.0)) return -1;
        const double nu = sqrt(nu2);
        if (fabs(sin(M_PI * nu)) < 1e-3) return -1;   /* Y_nu's formula needs non-integer nu */
        const double H2 = V / 3.0;
        const double complex A = 0.5 * sqrt(M_PI) * cexp(I * (nu + 0.5) * M_PI / 2.0);
        const double complex B = 0.5 * sqrt(M_PI) * cexp(I * (nu + 1.5) * M_PI / 2.0);
        const double complex alpha[2] = {A + B * cos(M_PI * nu) / sin(M_PI * nu), -B / sin(M_PI * nu)};
        const double mus[2] = {nu, -nu};
        double complex F = 0.0, G = 0.0;   /* F and -y F' */
        for (int k = 0; k < 2; ++k) {
            const double mu = mus[k];
            for (int m = 0; m < 30; ++m) {
                const double c = ((m % 2) ? -1.0 : 1.0) / (tgamma((double)m + 1.0) * tgamma((double)m + mu + 1.0) *
                                                            pow(2.0, 2.0 * m + mu));
                const double p = 2.0 * m + mu + 1.5;
                const double term = c * pow(sigma, p);
                F += alpha[k] * term;
                G -= alpha[k] * p * term;
            }
        }
        const double c = H2 / (2.0 * M_PI * M_PI);
        Xpp_out[j] = c * creal(F * conj(F));
        Xpq_out[j] = c * creal(F * conj(G));
        Xqq_out[j] = c * creal(G * conj(G));
    }
    return 0;
}

/* The symmetric positive semi-definite square root of [[a, b], [b, c]]:      */
/* S = (Xi + s 1)/t with s = sqrt(det Xi), t = sqrt(tr Xi + 2 s) (S^2 = Xi by  */
/* the Cayley-Hamilton identity Xi^2 - tr(Xi) Xi + det(Xi) 1 = 0); zero for   */
/* Xi = 0.  Returns -1 if Xi is not positive semi-definite.                   */
int orc_sqrt_sym2(double a, double b, double c, double *Spp, double *Spq, double *Sqq)
{
    const double det = a * c - b * b;
    if (!(a >= 0.0) || !(c >= 0.0) || !(det >= 0.0)) return -1;
    const double s = sqrt(det);
    const double tr = a + c + 2.0 * s;
    if (tr == 0.0) { *Spp = *Spq = *Sqq = 0.0; return 0; }
    const double t = sqrt(tr);
    *Spp = (a + s) / t;
    *Spq = b / t;
    *Sqq = (c + s) / t;
    return 0;
}

/* The two unit Gaussians (xi_1, xi_2) of step n with 2D noise: call m = n >> 1 */
/* of the generator gives (xi_1, xi_2) of step 2m from (u0, u1) and of step   */
/* 2m + 1 from (u2, u3) (same Box-Muller pairs as the 1D stream).              */
void orc_normals2d(uint64_t seed, uint32_t instance, uint64_t traj, uint64_t n0, uint64_t count, double *z_out)
{
    for (uint64_t i = 0; i < count; ++i) {
        const uint64_t n = n0 + i;
        double z[4];
        orc_four_normals(seed, instance, traj, n >> 1, z);
        z_out[2 * i] = z[2 * (n & 1)];
        z_out[2 * i + 1] = z[2 * (n & 1) + 1];
    }
}

typedef struct {
    int kind;
    double pot[7];
    int n_tab;
    double phi_lo, phi_hi;           /* node coordinates: phi, or the run's time N = n dN with tab_axis */
    int tab_axis;
    const double *Spp, *Spq, *Sqq;   /* square roots of the node covariances */
    const double *e1, *e2;           /* unit principal axis of the node covariances */
    double phi_in, pi_in, phi_end;
    int bias_kind;
    double A_bias;
    double dN;
    uint64_t seed;
    uint32_t instance;
    int64_t max_steps;
} orc_problem2d;

/* Unit eigenvector of [[a, b], [b, c]] (symmetric) for its largest eigenvalue        */
/* lambda = (a + c)/2 + r, r = sqrt(((a - c)/2)^2 + b^2), with a non-negative phi       */
/* component; (1, 0) when the eigenvalues coincide (b = 0, a = c) or the matrix is 0. */
void orc_principal_axis(double a, double b, double c, double *e1, double *e2)
{
    const double r = sqrt(0.25 * (a - c) * (a - c) + b * b);
    double v1, v2;
    if (a >= c) {            /* (lambda - c, b) */
        v1 = 0.5 * (a - c) + r;
        v2 = b;
    } else {                 /* (b, lambda - a) */
        v1 = b;
        v2 = 0.5 * (c - a) + r;
    }
    if (v1 < 0.0) { v1 = -v1; v2 = -v2; }
    const double norm = sqrt(v1 * v1 + v2 * v2);
    if (norm == 0.0) { *e1 = 1.0; *e2 = 0.0; return; }
    *e1 = v1 / norm;
    *e2 = v2 / norm;
}

/* S and e at the coordinate phi (or the time, for a time-indexed table): linear     */
/* interpolation of the nodes' square roots and principal axes, clamped to the edge  */
/* nodes.                                                                            */
static void orc_table2d_lookup(const orc_problem2d *P, double phi, double S[3], double e[2])
{
    if (P->n_tab == 1) {
        S[0] = P->Spp[0]; S[1] = P->Spq[0]; S[2] = P->Sqq[0];
        e[0] = P->e1[0]; e[1] = P->e2[0];
        return;
    }
    const double h = (P->phi_hi - P->phi_lo) / (double)(P->n_tab - 1);
    const double x = (phi - P->phi_lo) / h;
    double jf = floor(x);
    if (jf < 0.0) jf = 0.0;
    if (jf > (double)(P->n_tab - 2)) jf = (double)(P->n_tab - 2);
    const int j = (int)jf;
    double f = x - jf;
    if (f < 0.0) f = 0.0;
    if (f > 1.0) f = 1.0;
    S[0] = P->Spp[j] + f * (P->Spp[j + 1] - P->Spp[j]);
    S[1] = P->Spq[j] + f * (P->Spq[j + 1] - P->Spq[j]);
    S[2] = P->Sqq[j] + f * (P->Sqq[j + 1] - P->Sqq[j]);
    e[0] = P->e1[j] + f * (P->e1[j + 1] - P->e1[j]);
    e[1] = P->e2[j] + f * (P->e2[j + 1] - P->e2[j]);
}

/* One trajectory with 2D noise: eq. (full_langevin_equation) stepped with    */
/* eq. (euler_step_phi_and_pi) plus the bias, weight of eq. (weight_A) with    */
/* Xi = S^2.  The diffusion-based bias in 2D is B = A S e, e the unit principal */
/* axis of Xi (phi component >= 0), i.e. the push A along e in noise space:    */
/* in the rank-1 limit Xi = s s^T it is B = A s, the 1D bias of Sec. 4.1.       */
static void orc_trajectory2d(const orc_problem2d *P, uint64_t traj, double *N_out, double *lnw_out,
                             uint32_t *steps_out, double *phi2_out)
{
    const double dN = P->dN;
    const double sqrt_dN = sqrt(dN);
    double phi = P->phi_in, pi_ = P->pi_in, lnw = 0.0;
    int64_t n = 0;
    double zbuf[4];
    uint64_t zcall = UINT64_MAX;
    for (;;) {
        if (n >= P->max_steps) {
            *N_out = NAN;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n | ORC_FLAG_CENSORED;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi; }
            return;
        }
        const uint64_t call = (uint64_t)n >> 1;
        if (call != zcall) { orc_four_normals(P->seed, P->instance, traj, call, zbuf); zcall = call; }
        const double xi1 = zbuf[2 * (n & 1)], xi2 = zbuf[2 * (n & 1) + 1];
        /* drift vector D, eq. (full_langevin_equation) */
        const double V = orc_V(P->kind, P->pot, phi);
        const double dV = orc_dV(P->kind, P->pot, phi);
        const double D_phi = pi_;
        const double D_pi = -(3.0 - pi_ * pi_ / 2.0) * (pi_ + dV / V);
        /* noise matrix S, principal axis e, bias B = A S e */
        double S[3], e[2];
        orc_table2d_lookup(P, P->tab_axis ? (double)n * dN : phi, S, e);
        const double A = (P->bias_kind == ORC_BIAS_CONST) ? P->A_bias : 0.0;
        const double B_phi = A * (S[0] * e[0] + S[1] * e[1]);
        const double B_pi = A * (S[1] * e[0] + S[2] * e[1]);
        const double noise_phi = (S[0] * xi1 + S[1] * xi2) * sqrt_dN;
        const double noise_pi = (S[1] * xi1 + S[2] * xi2) * sqrt_dN;
        const double phi_next = phi + D_phi * dN + B_phi * dN + noise_phi;
        const double pi_next = pi_ + D_pi * dN + B_pi * dN + noise_pi;
        /* dA of eq. (weight_A), (B dN/2 + S xi sqrt(dN))^T Xi^-1 B with Xi = S S, evaluated as  */
        /* u . (u dN/2 + xi sqrt(dN)) with u = S^-1 B (S symmetric, so Xi^-1 = S^-1 S^-1)       */
        if (A != 0.0 && (S[0] != 0.0 || S[1] != 0.0 || S[2] != 0.0)) {
            const double detS = S[0] * S[2] - S[1] * S[1];
            const double u1 = (S[2] * B_phi - S[1] * B_pi) / detS;
            const double u2 = (S[0] * B_pi - S[1] * B_phi) / detS;
            const double dA = u1 * (u1 * dN / 2.0 + xi1 * sqrt_dN) + u2 * (u2 * dN / 2.0 + xi2 * sqrt_dN);
            lnw -= dA;
        }
        n += 1;
        if (phi_next <= P->phi_end) {
            const double frac = (phi - P->phi_end) / (phi - phi_next);
            *N_out = (double)(n - 1) * dN + dN * frac;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi_next; }
            return;
        }
        if (pi_next * pi_next / 2.0 >= 1.0) {
            *N_out = (double)n * dN;
            *lnw_out = lnw;
            *steps_out = (uint32_t)n | ORC_FLAG_ENDED_EARLY;
            if (phi2_out) { phi2_out[0] = phi; phi2_out[1] = phi_next; }
            return;
        }
        phi = phi_next;
        pi_ = pi_next;
    }
}

/* Trajectories traj_offset .. traj_offset + n_traj - 1 with 2D noise given by */
/* the node covariances Xi (each zero or positive definite).  bias_kind: NONE  */
/* or CONST.  tab_axis 1: the nodes are in the run's time (phi_lo, phi_hi hold */
/* N), read at N = n dN.  Returns 0, or -1 on invalid input.                   */
int orc_run2d(int kind, const double pot[7], int n_tab, double phi_lo, double phi_hi, const double *Xpp,
              const double *Xpq, const double *Xqq, int tab_axis, double phi_in, double pi_in, double phi_end,
              int bias_kind,
              double A_bias, double dN, uint64_t seed, uint32_t instance, uint64_t traj_offset, uint64_t n_traj,
              int64_t max_steps, double *N_out, double *lnw_out, uint32_t *steps_out, double *phi2_out,
              int n_threads)
{
    if (n_tab < 1 || !(dN > 0.0) || max_steps < 1 || max_steps > (int64_t)ORC_STEP_MASK) return -1;
    if (!(phi_in > phi_end)) return -1;
    if (bias_kind != ORC_BIAS_NONE && bias_kind != ORC_BIAS_CONST) return -1;
    double *S = (double *)malloc(sizeof(double) * 5 * (size_t)n_tab);
    if (!S) return -1;
    for (int j = 0; j < n_tab; ++j) {
        const double det = Xpp[j] * Xqq[j] - Xpq[j] * Xpq[j];
        const int zero = Xpp[j] == 0.0 && Xpq[j] == 0.0 && Xqq[j] == 0.0;
        if ((!zero && !(Xpp[j] > 0.0 && det > 0.0)) ||
            orc_sqrt_sym2(Xpp[j], Xpq[j], Xqq[j], &S[j], &S[n_tab + j], &S[2 * n_tab + j]) != 0) {
            free(S);
            return -1;
        }
        orc_principal_axis(Xpp[j], Xpq[j], Xqq[j], &S[3 * n_tab + j], &S[4 * n_tab + j]);
    }
    orc_problem2d P;
    memset(&P, 0, sizeof P);
    P.kind = kind;
    memcpy(P.pot, pot, sizeof P.pot);
    P.n_tab = n_tab; P.phi_lo = phi_lo; P.phi_hi = phi_hi; P.tab_axis = tab_axis;
    P.Spp = S; P.Spq = S + n_tab; P.Sqq = S + 2 * n_tab; P.e1 = S + 3 * n_tab; P.e2 = S + 4 * n_tab;
    P.phi_in = phi_in; P.pi_in = pi_in; P.phi_end = phi_end;
    P.bias_kind = bias_kind; P.A_bias = A_bias;
    P.dN = dN; P.seed = seed; P.instance = instance; P.max_steps = max_steps;
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    const int64_t nt = (int64_t)n_traj;
#pragma omp parallel for num_threads(n_thr) schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i)
        orc_trajectory2d(&P, traj_offset + (uint64_t)i, &N_out[i], &lnw_out[i], &steps_out[i],
                         phi2_out ? &phi2_out[2 * i] : NULL);
    free(S);
    return 0;
}

/* ========================================================================= */
/* Bessel-matched noise table (Sec. 3.4).                                     */
/* ========================================================================= */

/* J_mu(y) and y dJ_mu/dy by the power series; non-integer mu, y of order 1. */
static void orc_bessel_j_series(double mu, double y, double *J, double *yJp)
{
    double s = 0.0, sd = 0.0;
    for (int m = 0; m < 40; ++m) {
        const double p = 2.0 * m + mu;
        const double c = ((m % 2) ? -1.0 : 1.0) / (tgamma((double)m + 1.0) * tgamma((double)m + mu + 1.0)) *
                         pow(0.5 * y, p);
        s += c;
        sd += p * c;
    }
    *J = s;
    *yJp = sd;
}

/* Bessel coefficients of eq. (bessel_matching).  The mode is written as       */
/* delta phi_k = u / pref, u = A J_nu(y) + B Y_nu(y), y = -k eta, pref =        */
/* a/sqrt(-eta) (eq. delta_phi_bessel).  With d/dN y = -y and d/dN pref =       */
/* (3/2) pref (de Sitter, epsilon_1 << 1), the two conditions u = pref dphi,    */
/* du/dN = pref (3/2 dphi + d dphi/dN) give A and B by Cramer's rule.  Their    */
/* common denominator J dY/dN - Y dJ/dN is -y W[J_nu, Y_nu](y) = -2/pi, the     */
/* Wronskian of the Bessel functions, so B needs J_nu only and holds for every */
/* nu > 0.  A needs Y_nu = (J_nu cos nu pi - J_-nu)/sin nu pi and is NaN where */
/* |sin nu pi| < 1e-3.  dphi, ddphi, A, B are complex (re, im).                 */
void orc_bessel_match(double nu, double y, double pref, const double dphi[2], const double ddphi[2], double A[2],
                      double B[2])
{
    double Jn, yJn;
    orc_bessel_j_series(nu, y, &Jn, &yJn);
    const double dJ = -yJn;                                  /* d/dN of J_nu(y) */
    const double den = -2.0 / M_PI;
    const double complex f = dphi[0] + I * dphi[1], fp = ddphi[0] + I * ddphi[1];
    const double complex g = 1.5 * f + fp;                   /* (du/dN) / pref */
    const double complex b = -pref * (f * dJ - g * Jn) / den;
    B[0] = creal(b); B[1] = cimag(b);
    const double sn = sin(M_PI * nu), cn = cos(M_PI * nu);
    if (fabs(sn) < 1e-3) {
        A[0] = A[1] = NAN;
        return;
    }
    double Jm, yJm;
    orc_bessel_j_series(-nu, y, &Jm, &yJm);
    const double Y = (Jn * cn - Jm) / sn, dY = -(yJn * cn - yJm) / sn;
    const double complex a = pref * (f * dY - g * Y) / den;
    A[0] = creal(a); A[1] = cimag(a);
}

/* Background (phi, pi) and one Fourier mode in e-fold time.  The background    */
/* follows eq. (klein_gordon) with eq. (Friedmann), H^2 = V/(3 - eps1); the     */
/* mode follows eq. (full_delta_phi) divided by H^2:                            */
/*   dphi'' + (3 - eps1) dphi' + [k^2 e^(-2N)/H^2 + V''/H^2 - pi^2 (3 - eps1)   */
/*            - 2 pi pi'] dphi = 0,                                             */
/* where the last two terms are a^-3 d/dt(a^3 phidot^2/H) / H^2 and a = e^N.    */
/* On each side of the kink of the piecewise-linear potential V'' = 0; the      */
/* kink itself is handled in orc_mode_advance.                                  */
typedef struct { double phi, pi_, fr, fi, gr, gi; } orc_mode_state;   /* f = dphi, g = d dphi/dN */

/* `upper` evaluates the piecewise-linear potential on its phi >= phi_T branch */
/* (extended below phi_T), for the step that ends on the kink.                 */
static void orc_mode_rhs(int kind, const double pot[7], double k, double N, const orc_mode_state *s, int with_mode,
                         int upper, orc_mode_state *d)
{
    double V = orc_V(kind, pot, s->phi), dV = orc_dV(kind, pot, s->phi);
    if (upper && kind == ORC_POT_PIECEWISE_LINEAR) {
        V = pot[0] + pot[2] * (s->phi - pot[1]);
        dV = pot[2];
    }
    const double eps1 = 0.5 * s->pi_ * s->pi_;
    const double dpi = -(3.0 - eps1) * (s->pi_ + dV / V);
    d->phi = s->pi_;
    d->pi_ = dpi;
    if (!with_mode) { d->fr = d->fi = d->gr = d->gi = 0.0; return; }
    const double H2 = V / (3.0 - eps1);
    const double d2V = orc_d2V(kind, pot, s->phi);
    const double mass = k * k * exp(-2.0 * N) / H2 + d2V / H2 - s->pi_ * s->pi_ * (3.0 - eps1) - 2.0 * s->pi_ * dpi;
    d->fr = s->gr;
    d->fi = s->gi;
    d->gr = -(3.0 - eps1) * s->gr - mass * s->fr;
    d->gi = -(3.0 - eps1) * s->gi - mass * s->fi;
}

static void orc_mode_axpy(orc_mode_state *o, const orc_mode_state *s, const orc_mode_state *k, double c)
{
    o->phi = s->phi + c * k->phi; o->pi_ = s->pi_ + c * k->pi_;
    o->fr = s->fr + c * k->fr; o->fi = s->fi + c * k->fi;
    o->gr = s->gr + c * k->gr; o->gi = s->gi + c * k->gi;
}

/* One classical fourth-order Runge-Kutta step of size h. */
static void orc_mode_rk4(int kind, const double pot[7], double k, double N, double h, orc_mode_state *s, int with_mode,
                         int upper)
{
    orc_mode_state k1, k2, k3, k4, t;
    orc_mode_rhs(kind, pot, k, N, s, with_mode, upper, &k1);
    orc_mode_axpy(&t, s, &k1, 0.5 * h);
    orc_mode_rhs(kind, pot, k, N + 0.5 * h, &t, with_mode, upper, &k2);
    orc_mode_axpy(&t, s, &k2, 0.5 * h);
    orc_mode_rhs(kind, pot, k, N + 0.5 * h, &t, with_mode, upper, &k3);
    orc_mode_axpy(&t, s, &k3, h);
    orc_mode_rhs(kind, pot, k, N + h, &t, with_mode, upper, &k4);
    s->phi += h / 6.0 * (k1.phi + 2.0 * k2.phi + 2.0 * k3.phi + k4.phi);
    s->pi_ += h / 6.0 * (k1.pi_ + 2.0 * k2.pi_ + 2.0 * k3.pi_ + k4.pi_);
    s->fr += h / 6.0 * (k1.fr + 2.0 * k2.fr + 2.0 * k3.fr + k4.fr);
    s->fi += h / 6.0 * (k1.fi + 2.0 * k2.fi + 2.0 * k3.fi + k4.fi);
    s->gr += h / 6.0 * (k1.gr + 2.0 * k2.gr + 2.0 * k3.gr + k4.gr);
    s->gi += h / 6.0 * (k1.gi + 2.0 * k2.gi + 2.0 * k3.gi + k4.gi);
}

/* Advance from N to N_stop in RK4 steps of at most h_max and, with the mode   */
/* on, at most 1/200 of its oscillation period 2 pi aH/k.  With `kink` set and  */
/* the piecewise-linear potential, a step that would take phi from above the    */
/* kink phi_T to at or below it is shortened (by bisection of its size) to end  */
/* on phi_T, with every stage on the upper branch; there the delta function in V'' = (A_+ - A_-) delta(phi - phi_T)  */
/* changes d dphi/dN by -(A_+ - A_-) dphi / (H^2 |pi|) (its integral over N,    */
/* dN = dphi/|pi|), and phi is moved one ulp below phi_T.                      */
static void orc_mode_advance(int kind, const double pot[7], double k, double *N, double N_stop, orc_mode_state *s,
                             int with_mode, int kink, double h_max)
{
    const double phi_T = pot[1];
    while (*N < N_stop) {
        double h = fmin(h_max, N_stop - *N);
        if (with_mode) {
            const double aH = exp(*N) * sqrt(orc_V(kind, pot, s->phi) / (3.0 - 0.5 * s->pi_ * s->pi_));
            h = fmin(h, 2.0 * M_PI * aH / (800.0 * k));
        }
        orc_mode_state t = *s;
        orc_mode_rk4(kind, pot, k, *N, h, &t, with_mode, 0);
        if (!(kink && kind == ORC_POT_PIECEWISE_LINEAR && s->phi > phi_T && t.phi <= phi_T)) {
            *s = t;
            *N += h;
            continue;
        }
        double lo = 0.0, hi = h;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            orc_mode_state u = *s;
            orc_mode_rk4(kind, pot, k, *N, mid, &u, with_mode, 1);
            if (u.phi > phi_T) lo = mid; else hi = mid;
        }
        orc_mode_rk4(kind, pot, k, *N, hi, s, with_mode, 1);
        *N += hi;
        if (with_mode) {
            const double H2 = orc_V(kind, pot, phi_T) / (3.0 - 0.5 * s->pi_ * s->pi_);
            const double kick = -(pot[2] - pot[3]) / (H2 * fabs(s->pi_));
            s->gr += kick * s->fr;
            s->gi += kick * s->fi;
        }
        s->phi = nextafter(phi_T, -INFINITY);
    }
}

/* nu^2(phi) of eq. (nu_squared_approximation), and nu (NaN where nu^2 <= 0). */
static double orc_nu2_approx(int kind, const double pot[7], double phi)
{
    const double V = orc_V(kind, pot, phi);
    const double dVV = orc_dV(kind, pot, phi) / V, d2VV = orc_d2V(kind, pot, phi) / V;
    return 9.0 / 4.0 - 3.0 * (d2VV - dVV * dVV);
}

static double orc_nu_approx(int kind, const double pot[7], double phi)
{
    const double nu2 = orc_nu2_approx(kind, pot, phi);
    return nu2 > 0.0 ? sqrt(nu2) : NAN;
}

/* Classical trajectory from (phi_start, pi_start) at N = 0, sampled every 1e-4 e-folds (the  */
/* kink landed on exactly), until phi < phi_stop, N >= N_stop, eps1 >= 1 or N > 200.  When    */
/* phi_ref is finite, *N_ref receives the time the trajectory passes it (NaN if it does not   */
/* before stopping), and the sampling stops at N_ref + N_after instead of N_stop.  Returns    */
/* the sample count, or 0 on allocation failure (arrays freed).                             */
static void orc_hermite_root(const double *bN, const double *bphi, const double *bpi, size_t i, double target,
                             double *N_out, double *pi_out);

static size_t orc_background(int kind, const double pot[7], double phi_start, double pi_start, double phi_stop,
                             double N_stop, double phi_ref, double N_after, double *N_ref, double **bN_out,
                             double **bphi_out, double **bpi_out)
{
    const double hb = 1e-4;
    size_t cap = (size_t)1 << 16, nb = 0;
    double *bN = NULL, *bphi = NULL, *bpi = NULL;
    orc_mode_state s = {phi_start, pi_start, 0.0, 0.0, 0.0, 0.0};
    double N = 0.0;
    if (N_ref) *N_ref = NAN;
    for (;;) {
        if (nb == 0 || nb == cap) {
            if (nb) cap *= 2;
            double *a = (double *)realloc(bN, sizeof(double) * cap);
            if (a) bN = a;
            double *b = a ? (double *)realloc(bphi, sizeof(double) * cap) : NULL;
            if (b) bphi = b;
            double *c = b ? (double *)realloc(bpi, sizeof(double) * cap) : NULL;
            if (c) bpi = c;
            if (!a || !b || !c) { free(bN); free(bphi); free(bpi); return 0; }
        }
        bN[nb] = N; bphi[nb] = s.phi; bpi[nb] = s.pi_; ++nb;
        if (N_ref && isnan(*N_ref) && nb >= 2 && bphi[nb - 2] > phi_ref && bphi[nb - 1] <= phi_ref) {
            double pr;
            orc_hermite_root(bN, bphi, bpi, nb - 1, phi_ref, N_ref, &pr);
            N_stop = *N_ref + N_after;
        }
        if (s.phi < phi_stop || N >= N_stop || 0.5 * s.pi_ * s.pi_ >= 1.0 || N > 200.0) break;
        orc_mode_advance(kind, pot, 0.0, &N, N + hb, &s, 0, 1, hb);
    }
    *bN_out = bN; *bphi_out = bphi; *bpi_out = bpi;
    return nb;
}

/* The time at which phi(N) reaches target inside samples [i-1, i] (bphi[i-1] > target >= bphi[i]): */
/* the root of the cubic Hermite interpolant of phi, by Newton; pi there interpolated linearly.   */
static void orc_hermite_root(const double *bN, const double *bphi, const double *bpi, size_t i, double target,
                             double *N_out, double *pi_out)
{
    const double N0 = bN[i - 1], dn = bN[i] - bN[i - 1];
    const double p0 = bphi[i - 1], p1 = bphi[i], m0 = bpi[i - 1] * dn, m1 = bpi[i] * dn;
    double t = (p0 - target) / (p0 - p1);
    for (int it = 0; it < 50; ++it) {
        const double t2 = t * t, t3 = t2 * t;
        const double v = (2 * t3 - 3 * t2 + 1) * p0 + (t3 - 2 * t2 + t) * m0 + (-2 * t3 + 3 * t2) * p1 +
                         (t3 - t2) * m1 - target;
        const double dv = (6 * t2 - 6 * t) * p0 + (3 * t2 - 4 * t + 1) * m0 + (-6 * t2 + 6 * t) * p1 +
                          (3 * t2 - 2 * t) * m1;
        const double step = v / dv;
        t -= step;
        if (fabs(step) < 1e-16) break;
    }
    *N_out = N0 + t * dn;
    *pi_out = bpi[i - 1] + t * (bpi[i] - bpi[i - 1]);
}

/* 4|B_k|^2/pi of the mode that crosses k = sigma a H at N_sigma, where the classical trajectory */
/* is at (phi_j, pi_j).  The mode starts at the last sample with k >= 100 aH in the            */
/* Bunch-Davies state of eq. (bunch_davies), with the first correction of the Hankel            */
/* function's large-argument expansion, e^(i y)(1 + i c/y)/(a sqrt(2k)), c = (4 nu^2 - 1)/8,     */
/* y = k/(aH) (overall phase dropped).  It is evolved through eq. (full_delta_phi) to N_sigma   */
/* (taking the kink's kick when phi_j < phi_T) and matched by eq. (bessel_matching) with        */
/* nu = nu(phi_j) and -k eta = sigma.  Returns 0; -1 if the mode would have to start before    */
/* N = 0; -2 on a non-finite or zero result.                                                   */
static int orc_matched_factor(int kind, const double pot[7], double sigma, double phi_j, double pi_j, double Ns,
                              const double *bN, const double *bphi, const double *bpi, size_t nb, double *fac_out)
{
    const double Hs = sqrt(orc_V(kind, pot, phi_j) / (3.0 - 0.5 * pi_j * pi_j));
    const double k = sigma * exp(Ns) * Hs;
    const double aH0 = sqrt(orc_V(kind, pot, bphi[0]) / (3.0 - 0.5 * bpi[0] * bpi[0]));
    if (k < 100.0 * aH0) return -1;
    size_t i0 = 0;
    while (i0 + 1 < nb) {
        const double aH = exp(bN[i0 + 1]) * sqrt(orc_V(kind, pot, bphi[i0 + 1]) /
                                                 (3.0 - 0.5 * bpi[i0 + 1] * bpi[i0 + 1]));
        if (k < 100.0 * aH) break;
        ++i0;
    }
    orc_mode_state st = {bphi[i0], bpi[i0], 0.0, 0.0, 0.0, 0.0};
    double Nm = bN[i0];
    {
        const double a = exp(Nm);
        const double y = k / (a * sqrt(orc_V(kind, pot, st.phi) / (3.0 - 0.5 * st.pi_ * st.pi_)));
        const double c = (4.0 * orc_nu2_approx(kind, pot, st.phi) - 1.0) / 8.0;
        const double complex F = (1.0 + I * c / y) / (a * sqrt(2.0 * k));
        /* d/dN [e^(iy) (1 + ic/y) / a] e^(-iy) = [(-1 - iy)(1 + ic/y) + ic/y] / a */
        const double complex G = ((-1.0 - I * y) * (1.0 + I * c / y) + I * c / y) / (a * sqrt(2.0 * k));
        st.fr = creal(F); st.fi = cimag(F);
        st.gr = creal(G); st.gi = cimag(G);
    }
    orc_mode_advance(kind, pot, k, &Nm, Ns, &st, 1, phi_j < pot[1], 2.5e-4);
    const double nu_j = orc_nu_approx(kind, pot, phi_j);
    const double dphi[2] = {st.fr, st.fi}, ddphi[2] = {st.gr, st.gi};
    double A[2], B[2];
    /* a/sqrt(-eta) at -k eta = sigma: e^N sqrt(k/sigma) */
    orc_bessel_match(nu_j, sigma, exp(Nm) * sqrt(k / sigma), dphi, ddphi, A, B);
    const double fac = 4.0 * (B[0] * B[0] + B[1] * B[1]) / M_PI;
    if (!(fac > 0.0) || !isfinite(fac)) return -2;
    *fac_out = fac;
    return 0;
}

/* Bessel-matched 1D noise table, eq. (covariance_constant_nu_bessel_matched), on nodes in phi. */
/* For each node phi_j the classical trajectory from (phi_start, pi_start) reaches, N_sigma is   */
/* the time it passes phi_j; the node's noise is the Bunch-Davies table's (eq.                  */
/* covariance_constant_nu) times sqrt(4 |B_k|^2/pi) of orc_matched_factor; tan theta_n = nu -   */
/* 3/2 is unchanged.  Nodes the trajectory does not reach (at or above phi_start, or beyond     */
/* where it is followed: phi < phi_lo, eps1 >= 1 or N > 200) keep the factor 1.  A node below   */
/* the kink takes the kick; one at or above it stops before it.  fac_out[j] = 4 |B_k|^2/pi.     */
/* Returns 0; -1 on invalid input, on a node reached before its mode can start at k = 100 aH at */
/* N >= 0, or on a non-finite result.                                                          */
int orc_noise_table_matched(int kind, const double pot[7], double sigma, int n, double phi_lo, double phi_hi,
                            double phi_start, double pi_start, double *S_out, double *tan_out, double *fac_out,
                            int n_threads)
{
    if (orc_noise_table_bessel(kind, pot, sigma, n, phi_lo, phi_hi, S_out, tan_out) != 0) return -1;
    if (!(sigma > 0.0) || sigma > 2.0) return -1;
    const double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    double *bN, *bphi, *bpi;
    const size_t nb = orc_background(kind, pot, phi_start, pi_start, phi_lo, INFINITY, NAN, 0.0, NULL, &bN, &bphi,
                                     &bpi);
    if (nb == 0) return -1;
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    int bad = 0;
#pragma omp parallel for num_threads(n_thr) schedule(dynamic, 1)
    for (int j = 0; j < n; ++j) {
        fac_out[j] = 1.0;
        const double phi_j = phi_lo + (double)j * h;
        if (!(bphi[0] > phi_j)) continue;                     /* at or above the start */
        size_t i = 1;
        while (i < nb && bphi[i] > phi_j) ++i;
        if (i >= nb) continue;                                /* never reached */
        double Ns, pis, fac;
        orc_hermite_root(bN, bphi, bpi, i, phi_j, &Ns, &pis);
        if (orc_matched_factor(kind, pot, sigma, phi_j, pis, Ns, bN, bphi, bpi, nb, &fac) != 0) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        fac_out[j] = fac;
        S_out[j] *= sqrt(fac);
    }
    free(bN); free(bphi); free(bpi);
    return bad ? -1 : 0;
}

/* The classical trajectory at time Ns = N_ref + tau (samples bN, bphi, bpi): phi by the cubic  */
/* Hermite interpolant of the samples around Ns, pi linearly.  The node at tau = 0 is the      */
/* reference point itself: phi_ref exactly, so that a reference on the kink (phi_ref = phi_T)  */
/* keeps the node on the branch before it.  -1 if Ns lies outside the samples.                 */
static int orc_time_node(const double *bN, const double *bphi, const double *bpi, size_t nb, double tau, double Ns,
                         double phi_ref, double *phi_j, double *pi_j)
{
    if (!(Ns >= bN[0]) || !(Ns <= bN[nb - 1])) return -1;
    size_t i = 1;
    while (i < nb - 1 && bN[i] < Ns) ++i;              /* bN[i-1] <= Ns <= bN[i] */
    const double dn = bN[i] - bN[i - 1], t = (Ns - bN[i - 1]) / dn;
    const double t2 = t * t, t3 = t2 * t;
    *phi_j = tau == 0.0 ? phi_ref
                        : (2 * t3 - 3 * t2 + 1) * bphi[i - 1] + (t3 - 2 * t2 + t) * bpi[i - 1] * dn +
                              (-2 * t3 + 3 * t2) * bphi[i] + (t3 - t2) * bpi[i] * dn;
    *pi_j = bpi[i - 1] + t * (bpi[i] - bpi[i - 1]);
    return 0;
}

/* The same noise on nodes in time: node j is the time tau_j = t_lo + j (t_hi - t_lo)/(n - 1)  */
/* after the classical trajectory from (phi_start, pi_start) passes phi_ref (the run's phi_in), */
/* so that a run indexes it by its own time n dN -- the paper's scheme, noise precomputed along */
/* the classical trajectory and indexed by time (Sec. 4.1).  Node j takes phi_j, pi_j of the   */
/* trajectory at N_sigma = N_ref + tau_j (cubic Hermite interpolation of phi, linear of pi),   */
/* the Bunch-Davies node and nu at phi_j, and the factor of orc_matched_factor.  phi_out[j]     */
/* (if not NULL) receives phi_j.  Returns 0; -1 on invalid input, if the trajectory does not   */
/* pass phi_ref, if a node lies outside the followed trajectory, or as orc_noise_table_matched.  */
int orc_noise_table_matched_time(int kind, const double pot[7], double sigma, int n, double t_lo, double t_hi,
                                 double phi_start, double pi_start, double phi_ref, double *S_out, double *tan_out,
                                 double *fac_out, double *phi_out, int n_threads)
{
    if (n < 1 || !(sigma > 0.0) || sigma > 2.0) return -1;
    if (n > 1 && !(t_hi > t_lo)) return -1;
    if (!(phi_start > phi_ref)) return -1;
    const double h = (n > 1) ? (t_hi - t_lo) / (double)(n - 1) : 0.0;
    double *bN, *bphi, *bpi, N_ref;
    const size_t nb = orc_background(kind, pot, phi_start, pi_start, -INFINITY, INFINITY, phi_ref,
                                     (n > 1 ? t_hi : t_lo) + 2e-4, &N_ref, &bN, &bphi, &bpi);
    if (nb == 0) return -1;
    if (isnan(N_ref)) { free(bN); free(bphi); free(bpi); return -1; }
    const int n_thr = orc_threads(n_threads);
    (void)n_thr;
    int bad = 0;
#pragma omp parallel for num_threads(n_thr) schedule(dynamic, 1)
    for (int j = 0; j < n; ++j) {
        const double tau = t_lo + (double)j * h, Ns = N_ref + tau;
        fac_out[j] = NAN;
        double phi_j, pi_j;
        if (orc_time_node(bN, bphi, bpi, nb, tau, Ns, phi_ref, &phi_j, &pi_j) != 0) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        if (phi_out) phi_out[j] = phi_j;
        double fac;
        if (orc_noise_table_bessel(kind, pot, sigma, 1, phi_j, phi_j, &S_out[j], &tan_out[j]) != 0 ||
            orc_matched_factor(kind, pot, sigma, phi_j, pi_j, Ns, bN, bphi, bpi, nb, &fac) != 0) {
#pragma omp atomic write
            bad = 1;
            continue;
        }
        fac_out[j] = fac;
        S_out[j] *= sqrt(fac);
    }
    free(bN); free(bphi); free(bpi);
    return bad ? -1 : 0;
}

/* The 2D covariance of orc_noise_table_bessel2d on nodes in time (Sec. 4.1: the noise precomputed */
/* along the classical trajectory and read by the run's time): node j is tau_j = t_lo + j h after */
/* the trajectory from (phi_start, pi_start) passes phi_ref, and takes the covariance at the      */
/* trajectory's phi there (orc_time_node).  phi_out (may be NULL) receives those phi.  Returns 0,  */
/* or -1 on invalid input, a reference the trajectory does not pass, a node outside it, or a node  */
/* the covariance rejects.                                                                         */
int orc_noise_table_bessel2d_time(int kind, const double pot[7], double sigma, int n, double t_lo, double t_hi,
                                  double phi_start, double pi_start, double phi_ref, double *Xpp_out,
                                  double *Xpq_out, double *Xqq_out, double *phi_out)
{
    if (n < 1 || !(sigma > 0.0) || sigma > 2.0) return -1;
    if (n > 1 && !(t_hi > t_lo)) return -1;
    if (!(phi_start > phi_ref)) return -1;
    const double h = (n > 1) ? (t_hi - t_lo) / (double)(n - 1) : 0.0;
    double *bN, *bphi, *bpi, N_ref;
    const size_t nb = orc_background(kind, pot, phi_start, pi_start, -INFINITY, INFINITY, phi_ref,
                                     (n > 1 ? t_hi : t_lo) + 2e-4, &N_ref, &bN, &bphi, &bpi);
    if (nb == 0) return -1;
    int bad = isnan(N_ref);
    for (int j = 0; j < n && !bad; ++j) {
        const double tau = t_lo + (double)j * h, Ns = N_ref + tau;
        double phi_j, pi_j;
        if (orc_time_node(bN, bphi, bpi, nb, tau, Ns, phi_ref, &phi_j, &pi_j) != 0) {
            bad = 1;
            break;
        }
        if (phi_out) phi_out[j] = phi_j;
        bad = orc_noise_table_bessel2d(kind, pot, sigma, 1, phi_j, phi_j, &Xpp_out[j], &Xpq_out[j], &Xqq_out[j]) != 0;
    }
    free(bN); free(bphi); free(bpi);
    return bad ? -1 : 0;
}
