// fpt_table.hip -- the Bessel-matched noise table of eq. (covariance_constant_nu_bessel_matched)
// (Sec. 3.4): the classical trajectory, one Fourier mode per table node solved through
// eq. (full_delta_phi) from its Bunch-Davies state to the coarse-graining time, and the
// Bessel coefficient B_k of eq. (bessel_matching) that rescales the node's noise.
//
// Two kernels.  match_background_kernel is one thread: the classical trajectory is a
// sequential ODE.  It writes a sample every kBgStep e-folds and, for every node, the index
// of the first sample at or below it.  match_node_kernel is one thread per node: each
// mode is an independent ODE solve of some 10^4 RK4 steps, all in FP64.
#include "internal.hpp"
#include "noise_node.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace fpt {

namespace {

constexpr double kBgStep = 1e-4;         // e-folds between trajectory samples
constexpr double kBgMaxN = 200.0;        // the trajectory is followed at most this long
constexpr double kModeMaxStep = 2.5e-4;  // largest RK4 step of a mode, in e-folds
constexpr double kStepsPerPeriod = 800.0;
constexpr double kStartRatio = 100.0;    // a mode starts at k = 100 aH

using Pot = PotParams;

// The RK4 step that ends on the kink of the piecewise-linear potential is evaluated on the
// upper branch (pot_eval's `upper`).

__device__ inline double hubble2(const Pot &p, double phi, double pi_)
{
    double V, dV, d2V;
    pot_eval(p, phi, false, V, dV, d2V);
    return V / (3.0 - 0.5 * pi_ * pi_);
}

// nu^2 of eq. (nu_squared_approximation).
__device__ inline double nu2_of(const Pot &p, double phi)
{
    double V, dV, d2V;
    pot_eval(p, phi, false, V, dV, d2V);
    const double r1 = dV / V;
    return 2.25 - 3.0 * (d2V / V - r1 * r1);
}

// Background (phi, pi) and, with MODE, the mode dphi = (fr, fi) and d dphi/dN = (gr, gi).
struct St {
    double phi, pi_, fr, fi, gr, gi;
};

// Time derivative in N.  Background: eq. (klein_gordon) in e-folds with H^2 = V/(3 - eps1)
// from eq. (Friedmann).  Mode: eq. (full_delta_phi) over H^2, whose last term,
// a^-3 d/dt(a^3 phidot^2/H), is H^2 (pi^2 (3 - eps1) + 2 pi dpi/dN).  kk = k^2.
template <bool MODE>
__device__ inline St deriv(const Pot &p, double kk, double N, const St &s, bool upper)
{
    double V, dV, d2V;
    pot_eval(p, s.phi, upper, V, dV, d2V);
    const double q = 3.0 - 0.5 * s.pi_ * s.pi_;
    const double dpi = -q * (s.pi_ + dV / V);
    St d;
    d.phi = s.pi_;
    d.pi_ = dpi;
    if (MODE) {
        const double inv_H2 = q / V;
        const double m2 = (kk * exp(-2.0 * N) + d2V) * inv_H2 - s.pi_ * (s.pi_ * q + 2.0 * dpi);
        d.fr = s.gr;
        d.fi = s.gi;
        d.gr = -q * s.gr - m2 * s.fr;
        d.gi = -q * s.gi - m2 * s.fi;
    } else {
        d.fr = d.fi = d.gr = d.gi = 0.0;
    }
    return d;
}

__device__ inline St axpy(const St &s, const St &k, double c)
{
    return St{s.phi + c * k.phi, s.pi_ + c * k.pi_, s.fr + c * k.fr, s.fi + c * k.fi, s.gr + c * k.gr,
              s.gi + c * k.gi};
}

template <bool MODE>
__device__ inline St rk4(const Pot &p, double kk, double N, double h, const St &s, bool upper)
{
    const St k1 = deriv<MODE>(p, kk, N, s, upper);
    const St k2 = deriv<MODE>(p, kk, N + 0.5 * h, axpy(s, k1, 0.5 * h), upper);
    const St k3 = deriv<MODE>(p, kk, N + 0.5 * h, axpy(s, k2, 0.5 * h), upper);
    const St k4 = deriv<MODE>(p, kk, N + h, axpy(s, k3, h), upper);
    const double c = h / 6.0;
    St o;
    o.phi = s.phi + c * (k1.phi + 2.0 * (k2.phi + k3.phi) + k4.phi);
    o.pi_ = s.pi_ + c * (k1.pi_ + 2.0 * (k2.pi_ + k3.pi_) + k4.pi_);
    o.fr = s.fr + c * (k1.fr + 2.0 * (k2.fr + k3.fr) + k4.fr);
    o.fi = s.fi + c * (k1.fi + 2.0 * (k2.fi + k3.fi) + k4.fi);
    o.gr = s.gr + c * (k1.gr + 2.0 * (k2.gr + k3.gr) + k4.gr);
    o.gi = s.gi + c * (k1.gi + 2.0 * (k2.gi + k3.gi) + k4.gi);
    return o;
}

// Integrate from *N to N_stop.  Steps: at most h_max and, with MODE, at most 1/800 of the
// mode's period 2 pi aH/k.  With `kink` (piecewise-linear potential), the step that would
// take phi from above phi_T to at or below it is cut, by bisection of its length, to end on
// phi_T; the delta function (A_+ - A_-) delta(phi - phi_T) in V'' then adds
// -(A_+ - A_-) dphi/(H^2 |pi|) to d dphi/dN, and phi continues one ulp below phi_T.
template <bool MODE>
__device__ void advance(const Pot &p, double k, double &N, double N_stop, St &s, bool kink, double h_max)
{
    const double kk = k * k;
    const bool has_kink = kink && p.kind == kPotPiecewiseLinear;
    while (N < N_stop) {
        double h = fmin(h_max, N_stop - N);
        if (MODE) h = fmin(h, (2.0 * M_PI / kStepsPerPeriod) * exp(N) * sqrt(hubble2(p, s.phi, s.pi_)) / k);
        const St t = rk4<MODE>(p, kk, N, h, s, false);
        if (!(has_kink && s.phi > p.phi_T && t.phi <= p.phi_T)) {
            s = t;
            N += h;
            continue;
        }
        double lo = 0.0, hi = h;
        for (int it = 0; it < 64; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (rk4<MODE>(p, kk, N, mid, s, true).phi > p.phi_T) lo = mid;
            else hi = mid;
        }
        s = rk4<MODE>(p, kk, N, hi, s, true);
        N += hi;
        if (MODE) {
            double V, dV, d2V;
            pot_eval(p, p.phi_T, true, V, dV, d2V);
            const double H2 = V / (3.0 - 0.5 * s.pi_ * s.pi_);
            const double kick = -(p.Ap - p.Am) / (H2 * fabs(s.pi_));
            s.gr += kick * s.fr;
            s.gi += kick * s.fi;
        }
        s.phi = nextafter(p.phi_T, -INFINITY);
    }
}

// J_mu(y) and y J_mu'(y) by the power series, each term from the previous one:
// t_m = t_{m-1} (-(y/2)^2) / (m (m + mu)),  t_0 = (y/2)^mu / Gamma(mu + 1).
__device__ inline void bessel_j(double mu, double y, double &J, double &yJp)
{
    const double q = -0.25 * y * y;
    double t = pow(0.5 * y, mu) / tgamma(mu + 1.0);
    double s = t, sd = mu * t;
    for (int m = 1; m < 40; ++m) {
        t *= q / ((double)m * ((double)m + mu));
        s += t;
        sd += (2.0 * m + mu) * t;
    }
    J = s;
    yJp = sd;
}

__global__ void match_background_kernel(Pot p, double phi_start, double pi_start, double phi_lo, double h_node,
                                        int n, double *bN, double *bphi, double *bpi, int cap, int *nb_out,
                                        int *first_idx)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    St s{phi_start, pi_start, 0.0, 0.0, 0.0, 0.0};
    double N = 0.0;
    int nb = 0;
    for (;;) {
        bN[nb] = N;
        bphi[nb] = s.phi;
        bpi[nb] = s.pi_;
        if (nb > 0) {
            // nodes first reached by this sample: bphi[nb] <= phi_j < bphi[nb-1] and phi_j < bphi[0]
            const double hi_phi = fmin(bphi[nb - 1], bphi[0]);
            if (s.phi < hi_phi) {
                int j0 = 0, j1 = n - 1;
                if (h_node > 0.0) {   // candidate range, clamped in FP64 before the conversion
                    const double a = fmin(fmax(floor((s.phi - phi_lo) / h_node) - 1.0, 0.0), (double)n);
                    const double b = fmin(fmax(ceil((hi_phi - phi_lo) / h_node) + 1.0, -1.0), (double)(n - 1));
                    j0 = (int)a;
                    j1 = (int)b;
                }
                for (int j = j0; j <= j1; ++j) {
                    const double pj = grid_node(phi_lo, j, h_node);
                    if (s.phi <= pj && pj < hi_phi && first_idx[j] < 0) first_idx[j] = nb;
                }
            }
        }
        ++nb;
        if (s.phi < phi_lo || 0.5 * s.pi_ * s.pi_ >= 1.0 || N > kBgMaxN || nb == cap) break;
        advance<false>(p, 0.0, N, N + kBgStep, s, true, kBgStep);
    }
    *nb_out = nb;
}

// The Bunch-Davies node of eq. (covariance_constant_nu) at phi: sqrt(Xi_phiphi), nu.  False where
// V <= 0 or nu^2 <= 0.
__device__ inline bool bd_node(const Pot &p, double sigma, double phi, double &S_bd, double &nu, double &V)
{
    double dV, d2V;
    pot_eval(p, phi, false, V, dV, d2V);
    const double nu2 = nu2_of(p, phi);
    if (!(V > 0.0) || !(nu2 > 0.0)) return false;
    nu = sqrt(nu2);
    S_bd = sqrt(V / 3.0) / (2.0 * M_PI) * (tgamma(nu) / (0.5 * sqrt(M_PI))) * pow(0.5 * sigma, 1.5 - nu);
    return true;
}

// 4|B_k|^2/pi of the mode that crosses k = sigma a H at N_sigma = Ns, where the classical trajectory
// is at (phi_j, pis) with V = V(phi_j) and nu = nu(phi_j).  Status bits: 2 (the mode would start
// before N = 0), 4 (non-finite or zero B_k); the factor is then NaN.
__device__ double matched_factor(const Pot &p, double sigma, double phi_j, double pis, double Ns, double V, double nu,
                                 const double *bN, const double *bphi, const double *bpi, int nb, int *status)
{
    const double k = sigma * exp(Ns) * sqrt(V / (3.0 - 0.5 * pis * pis));
    // start at the last sample with k >= 100 aH (aH grows while eps1 < 1)
    auto aH = [&](int ii) { return exp(bN[ii]) * sqrt(hubble2(p, bphi[ii], bpi[ii])); };
    if (k < kStartRatio * aH(0)) {
        atomicOr(status, 2);
        return NAN;
    }
    int lo = 0, hi = nb;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (k < kStartRatio * aH(mid)) hi = mid;
        else lo = mid;
    }
    double N = bN[lo];
    St s{bphi[lo], bpi[lo], 0.0, 0.0, 0.0, 0.0};
    {
        // Bunch-Davies: e^(iy)(1 + i c/y)/(a sqrt(2k)), c = (4 nu^2 - 1)/8, y = k/(aH), overall phase
        // dropped; d/dN of it is [(-1 - iy)(1 + ic/y) + ic/y]/(a sqrt(2k))
        const double a = exp(N);
        const double y = k / (a * sqrt(hubble2(p, s.phi, s.pi_)));
        const double c = (4.0 * nu2_of(p, s.phi) - 1.0) * 0.125;
        const double amp = 1.0 / (a * sqrt(2.0 * k));
        s.fr = amp;
        s.fi = amp * c / y;
        s.gr = amp * (-1.0 + c);        // Re[(-1 - iy)(1 + ic/y) + ic/y]
        s.gi = amp * (-y);              // Im[...] = -c/y - y + c/y
    }
    advance<true>(p, k, N, Ns, s, phi_j < p.phi_T, kModeMaxStep);
    // eq. (bessel_matching) at -k eta = sigma with nu(phi_j); a/sqrt(-eta) = e^N sqrt(k/sigma).  The
    // denominator J_nu dY_nu/dN - Y_nu dJ_nu/dN is -y W[J_nu, Y_nu](y) = -2/pi (the Bessel Wronskian),
    // so B_k = (pi/2) pref (dphi dJ/dN - g J) with g = 3/2 dphi + d dphi/dN, for every nu > 0.
    double Jn, yJn;
    bessel_j(nu, sigma, Jn, yJn);
    const double dJ = -yJn;
    const double pref = exp(N) * sqrt(k / sigma);
    const double g_r = 1.5 * s.fr + s.gr, g_i = 1.5 * s.fi + s.gi;
    const double b_r = 0.5 * M_PI * pref * (s.fr * dJ - g_r * Jn);
    const double b_i = 0.5 * M_PI * pref * (s.fi * dJ - g_i * Jn);
    const double fac = 4.0 * (b_r * b_r + b_i * b_i) / M_PI;
    if (!(fac > 0.0) || !isfinite(fac)) {
        atomicOr(status, 4);
        return NAN;
    }
    return fac;
}

// The time at which phi(N) reaches target inside samples [i-1, i]: Newton on the cubic Hermite
// interpolant of phi; pi there interpolated linearly.
__device__ inline void hermite_root(const double *bN, const double *bphi, const double *bpi, int i, double target,
                                    double &Ns, double &pis)
{
    const double dn = bN[i] - bN[i - 1];
    const double p0 = bphi[i - 1], p1 = bphi[i], m0 = bpi[i - 1] * dn, m1 = bpi[i] * dn;
    double t = (p0 - target) / (p0 - p1);
    for (int it = 0; it < 50; ++it) {
        const double t2 = t * t, t3 = t2 * t;
        const double v = (2.0 * t3 - 3.0 * t2 + 1.0) * p0 + (t3 - 2.0 * t2 + t) * m0 + (3.0 * t2 - 2.0 * t3) * p1 +
                         (t3 - t2) * m1 - target;
        const double dv = 6.0 * (t2 - t) * (p0 - p1) + (3.0 * t2 - 4.0 * t + 1.0) * m0 + (3.0 * t2 - 2.0 * t) * m1;
        const double step = v / dv;
        t -= step;
        if (fabs(step) < 1e-16) break;
    }
    Ns = bN[i - 1] + t * dn;
    pis = bpi[i - 1] + t * (bpi[i] - bpi[i - 1]);
}

__global__ void match_node_kernel(Pot p, double sigma, int n, double phi_lo, double h_node, const double *bN,
                                  const double *bphi, const double *bpi, const int *nb_ptr, const int *first_idx,
                                  double *S, double *tan_out, double *fac_out, int *status)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double phi_j = grid_node(phi_lo, j, h_node);
    double S_bd, nu, V;
    if (!bd_node(p, sigma, phi_j, S_bd, nu, V)) {
        atomicOr(status, 1);
        S[j] = tan_out[j] = fac_out[j] = 0.0;
        return;
    }
    tan_out[j] = nu - 1.5;
    double fac = 1.0;
    const int i = first_idx[j];
    if (i > 0) {
        double Ns, pis;
        hermite_root(bN, bphi, bpi, i, phi_j, Ns, pis);
        fac = matched_factor(p, sigma, phi_j, pis, Ns, V, nu, bN, bphi, bpi, *nb_ptr, status);
    }
    fac_out[j] = fac;
    S[j] = S_bd * sqrt(fac);
}

// Time nodes: the classical trajectory as in match_background_kernel, with the time N_ref at which
// it passes phi_ref (NaN if it does not); it is followed until N_ref + N_after once that is known.
__global__ void match_background_time_kernel(Pot p, double phi_start, double pi_start, double phi_ref, double N_after,
                                             double *bN, double *bphi, double *bpi, int cap, int *nb_out,
                                             double *N_ref_out)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    St s{phi_start, pi_start, 0.0, 0.0, 0.0, 0.0};
    double N = 0.0, N_ref = NAN, N_stop = INFINITY;
    int nb = 0;
    for (;;) {
        bN[nb] = N;
        bphi[nb] = s.phi;
        bpi[nb] = s.pi_;
        ++nb;
        if (isnan(N_ref) && nb >= 2 && bphi[nb - 2] > phi_ref && bphi[nb - 1] <= phi_ref) {
            double pr;
            hermite_root(bN, bphi, bpi, nb - 1, phi_ref, N_ref, pr);
            N_stop = N_ref + N_after;
        }
        if (N >= N_stop || 0.5 * s.pi_ * s.pi_ >= 1.0 || N > kBgMaxN || nb == cap) break;
        advance<false>(p, 0.0, N, N + kBgStep, s, true, kBgStep);
    }
    *nb_out = nb;
    *N_ref_out = N_ref;
}

// The trajectory at N_sigma = N_ref + tau (tau = t_lo + j h, formed without a fused multiply-add):
// phi by the cubic Hermite interpolant of the samples, pi linearly; tau = 0 is the reference point,
// phi_ref exactly (on a kink at phi_ref, the branch before it).  False where the trajectory does
// not pass phi_ref (N_ref NaN) or N_sigma lies outside the followed samples.
__device__ inline bool time_node(double t_lo, int j, double h, double phi_ref, const double *bN, const double *bphi,
                                 const double *bpi, int nb, double N_ref, double &Ns, double &phi_j, double &pi_j)
{
    const double tau = grid_node(t_lo, j, h);
    Ns = N_ref + tau;
    if (!(Ns >= bN[0]) || !(Ns <= bN[nb - 1]) || nb < 2) return false;
    // first sample at or after Ns (from 1, at most nb - 1)
    int lo = 0, hi = nb - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bN[mid] < Ns) lo = mid;
        else hi = mid;
    }
    const int i = hi;
    const double dn = bN[i] - bN[i - 1], t = (Ns - bN[i - 1]) / dn;
    const double t2 = t * t, t3 = t2 * t;
    phi_j = tau == 0.0 ? phi_ref
                       : (2.0 * t3 - 3.0 * t2 + 1.0) * bphi[i - 1] + (t3 - 2.0 * t2 + t) * bpi[i - 1] * dn +
                             (3.0 * t2 - 2.0 * t3) * bphi[i] + (t3 - t2) * bpi[i] * dn;
    pi_j = bpi[i - 1] + t * (bpi[i] - bpi[i - 1]);
    return true;
}

// Node j at N_sigma = N_ref + t_lo + j h: the trajectory's phi_j and pi_j there (time_node), the
// Bunch-Davies node and the factor.  Status 16: the trajectory does not pass phi_ref, or the node
// lies outside the followed trajectory.
__global__ void match_node_time_kernel(Pot p, double sigma, int n, double t_lo, double h, double phi_ref,
                                       const double *bN, const double *bphi, const double *bpi, const int *nb_ptr,
                                       const double *N_ref_ptr, double *S, double *tan_out, double *fac_out,
                                       double *phi_out, int *status)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int nb = *nb_ptr;
    S[j] = tan_out[j] = fac_out[j] = phi_out[j] = NAN;
    double Ns, phi_j, pi_j;
    if (!time_node(t_lo, j, h, phi_ref, bN, bphi, bpi, nb, *N_ref_ptr, Ns, phi_j, pi_j)) {
        atomicOr(status, 16);
        return;
    }
    phi_out[j] = phi_j;
    double S_bd, nu, V;
    if (!bd_node(p, sigma, phi_j, S_bd, nu, V)) {
        atomicOr(status, 1);
        return;
    }
    tan_out[j] = nu - 1.5;
    const double fac = matched_factor(p, sigma, phi_j, pi_j, Ns, V, nu, bN, bphi, bpi, nb, status);
    fac_out[j] = fac;
    S[j] = S_bd * sqrt(fac);
}

// 2D node j in time: the covariance of noise_node.hpp at the trajectory's phi there.  Status 16 as
// above, 1 where the covariance rejects the node.
__global__ void bessel2d_time_node_kernel(Pot p, double sigma, int n, double t_lo, double h, double phi_ref,
                                          const double *bN, const double *bphi, const double *bpi,
                                          const int *nb_ptr, const double *N_ref_ptr, double *Xpp, double *Xpq,
                                          double *Xqq, double *phi_out, int *status)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    Xpp[j] = Xpq[j] = Xqq[j] = phi_out[j] = NAN;
    double Ns, phi_j, pi_j;
    if (!time_node(t_lo, j, h, phi_ref, bN, bphi, bpi, *nb_ptr, *N_ref_ptr, Ns, phi_j, pi_j)) {
        atomicOr(status, 16);
        return;
    }
    phi_out[j] = phi_j;
    if (!bessel2d_node(p, sigma, phi_j, Xpp[j], Xpq[j], Xqq[j])) atomicOr(status, 1);
}

}  // namespace

size_t matched_scratch_bytes(int n) { return (size_t)kMatchCap * 3 * sizeof(double) + (size_t)(n + 2) * sizeof(int); }

hipError_t matched_table_launch(const PotParams &p, double sigma, int n, double phi_lo, double h_node,
                                double phi_start, double pi_start, void *scratch, double *d_S, double *d_tan,
                                double *d_fac, int *d_status, hipStream_t stream)
{
    double *bN = static_cast<double *>(scratch);
    double *bphi = bN + kMatchCap, *bpi = bphi + kMatchCap;
    int *nb = reinterpret_cast<int *>(bpi + kMatchCap);
    int *first_idx = nb + 1;
    hipError_t e = hipMemsetAsync(first_idx, 0xff, sizeof(int) * n, stream);   // -1: not reached
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(match_background_kernel, dim3(1), dim3(64), 0, stream, p, phi_start, pi_start, phi_lo,
                       h_node, n, bN, bphi, bpi, (int)kMatchCap, nb, first_idx);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(match_node_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, sigma, n, phi_lo, h_node,
                       bN, bphi, bpi, nb, first_idx, d_S, d_tan, d_fac, d_status);
    return hipGetLastError();
}

size_t matched_time_scratch_bytes() { return (size_t)kMatchCap * 3 * sizeof(double) + 16; }

hipError_t matched_time_launch(const PotParams &p, double sigma, int n, double t_lo, double h, double phi_start,
                               double pi_start, double phi_ref, double N_after, void *scratch, double *d_S,
                               double *d_tan, double *d_fac, double *d_phi, int *d_status, hipStream_t stream)
{
    double *bN = static_cast<double *>(scratch);
    double *bphi = bN + kMatchCap, *bpi = bphi + kMatchCap;
    int *nb = reinterpret_cast<int *>(bpi + kMatchCap);
    double *N_ref = reinterpret_cast<double *>(bpi + kMatchCap) + 1;
    hipLaunchKernelGGL(match_background_time_kernel, dim3(1), dim3(64), 0, stream, p, phi_start, pi_start, phi_ref,
                       N_after, bN, bphi, bpi, (int)kMatchCap, nb, N_ref);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(match_node_time_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, sigma, n, t_lo, h,
                       phi_ref, bN, bphi, bpi, nb, N_ref, d_S, d_tan, d_fac, d_phi, d_status);
    return hipGetLastError();
}

hipError_t bessel2d_time_launch(const PotParams &p, double sigma, int n, double t_lo, double h, double phi_start,
                                double pi_start, double phi_ref, double N_after, void *scratch, double *d_Xpp,
                                double *d_Xpq, double *d_Xqq, double *d_phi, int *d_status, hipStream_t stream)
{
    double *bN = static_cast<double *>(scratch);
    double *bphi = bN + kMatchCap, *bpi = bphi + kMatchCap;
    int *nb = reinterpret_cast<int *>(bpi + kMatchCap);
    double *N_ref = reinterpret_cast<double *>(bpi + kMatchCap) + 1;
    hipLaunchKernelGGL(match_background_time_kernel, dim3(1), dim3(64), 0, stream, p, phi_start, pi_start, phi_ref,
                       N_after, bN, bphi, bpi, (int)kMatchCap, nb, N_ref);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bessel2d_time_node_kernel, dim3((n + 63) / 64), dim3(64), 0, stream, p, sigma, n, t_lo, h,
                       phi_ref, bN, bphi, bpi, nb, N_ref, d_Xpp, d_Xpq, d_Xqq, d_phi, d_status);
    return hipGetLastError();
}

}  // namespace fpt
