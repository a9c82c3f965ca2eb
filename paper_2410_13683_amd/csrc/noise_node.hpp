// noise_node.hpp -- the 2D noise covariance of one table node, shared by the phi-node and
// time-node table kernels.
//
// Eq. (covariance_matrix_direct) from the full Bunch-Davies mode of eq. (delta_phi_bessel) at
// -k eta = sigma: with y = -k eta, delta phi_k = H k^(-3/2) F(y), F = y^(3/2) (A J_nu + B Y_nu),
// delta pi_k = H k^(-3/2) (-y F'(y)), so Xi = H^2/(2 pi^2) [[|F|^2, Re(F conj G)], [., |G|^2]]
// with G = -y F'.  Y_nu = (J_nu cos nu pi - J_-nu)/sin nu pi turns F into alpha_+ y^(3/2) J_nu +
// alpha_- y^(3/2) J_-nu, each J_mu summed as its power series (30 terms: below 1e-40 of the
// leading term for sigma <= 2).  nu^2 = 9/4 - 3 (V''/V - (V'/V)^2) and H^2 = V/3 as for the 1D
// table.
#pragma once

#include "potential.hpp"

#include <hip/hip_runtime.h>

#include <cmath>

namespace fpt {

struct Cplx {
    double re, im;
};
__device__ __forceinline__ Cplx cscale(Cplx a, double s) { return {a.re * s, a.im * s}; }
__device__ __forceinline__ Cplx cadd(Cplx a, Cplx b) { return {a.re + b.re, a.im + b.im}; }

// Xi at phi; false (and zeros) where V <= 0, nu^2 <= 0 or nu is within 1e-3 of an integer (the
// Y_nu form above needs sin nu pi away from 0).
__device__ inline bool bessel2d_node(const PotParams &pp, double sigma, double phi, double &Xpp, double &Xpq,
                                     double &Xqq)
{
    double V, dV, d2V;
    pot_eval(pp, phi, false, V, dV, d2V);
    const double r1 = dV / V, r2 = d2V / V;
    const double nu2 = 2.25 - 3.0 * (r2 - r1 * r1);
    const double nu = nu2 > 0.0 ? sqrt(nu2) : 0.0;
    double sn, cs;
    sincospi(nu, &sn, &cs);
    if (!(V > 0.0) || !(nu2 > 0.0) || fabs(sn) < 1e-3) {
        Xpp = Xpq = Xqq = 0.0;
        return false;
    }
    // A_k, B_k of eq. (A_k_and_B_k): sqrt(pi)/2 exp(i (nu + 1/2) pi/2), sqrt(pi)/2 exp(i (nu + 3/2) pi/2)
    const double hs = 0.5 * sqrt(M_PI);
    double sa, ca, sb, cb;
    sincospi(0.5 * (nu + 0.5), &sa, &ca);
    sincospi(0.5 * (nu + 1.5), &sb, &cb);
    const Cplx Ak = {hs * ca, hs * sa}, Bk = {hs * cb, hs * sb};
    const Cplx alpha[2] = {cadd(Ak, cscale(Bk, cs / sn)), cscale(Bk, -1.0 / sn)};
    const double mus[2] = {nu, -nu};
    Cplx F = {0.0, 0.0}, G = {0.0, 0.0};
    for (int k = 0; k < 2; ++k) {
        const double mu = mus[k];
        for (int m = 0; m < 30; ++m) {
            const double p = 2.0 * m + mu + 1.5;
            const double term = ((m & 1) ? -1.0 : 1.0) * pow(sigma, p) /
                                (tgamma((double)m + 1.0) * tgamma((double)m + mu + 1.0) * pow(2.0, 2.0 * m + mu));
            F = cadd(F, cscale(alpha[k], term));
            G = cadd(G, cscale(alpha[k], -p * term));
        }
    }
    const double c = (V / 3.0) / (2.0 * M_PI * M_PI);
    Xpp = c * (F.re * F.re + F.im * F.im);
    Xpq = c * (F.re * G.re + F.im * G.im);      // Re(F conj(G))
    Xqq = c * (G.re * G.re + G.im * G.im);
    return true;
}

}  // namespace fpt
