// potential.hpp -- V, V' and V'' of the library's potentials, for the noise-table
// generators (host and device).  The Euler-Maruyama kernels use their own forms of
// V'/V, written for the step (fpt_em.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace fpt {

// kind 0: piecewise linear, eq. (potential_starobinsky): V = V0 + A_+-(phi - phi_T),
//         the A_+ branch at phi >= phi_T;
// kind 1: exponential, V = V0 exp(A_+ (phi - phi_T));
// kind 2: Gaussian bump, eq. (potential_swagat): V = V0 u (1 + g), u = phi^2/(m^2 + phi^2),
//         g = K exp(-x^2/2), x = (phi - phi_T)/Sigma (phi_T is the bump's centre phi_0).
struct PotParams {
    int kind;
    double V0, phi_T, Ap, Am, m, K, Sigma;
};

// `upper` evaluates the piecewise-linear potential on its phi >= phi_T branch, continued
// below phi_T (other kinds ignore it).
__host__ __device__ inline void pot_eval(const PotParams &p, double phi, bool upper, double &V, double &dV,
                                         double &d2V)
{
    if (p.kind == 1) {
        V = p.V0 * exp(p.Ap * (phi - p.phi_T));
        dV = p.Ap * V;
        d2V = p.Ap * dV;
    } else if (p.kind == 2) {
        const double m2 = p.m * p.m, q = m2 + phi * phi, iq = 1.0 / q;
        const double u = phi * phi * iq;
        const double du = 2.0 * m2 * phi * iq * iq;
        const double d2u = 2.0 * m2 * (m2 - 3.0 * phi * phi) * iq * iq * iq;
        const double x = (phi - p.phi_T) / p.Sigma;
        const double g = p.K * exp(-0.5 * x * x);
        const double dg = -x / p.Sigma * g;
        const double d2g = (x * x - 1.0) / (p.Sigma * p.Sigma) * g;
        V = p.V0 * u * (1.0 + g);
        dV = p.V0 * (du * (1.0 + g) + u * dg);
        d2V = p.V0 * (d2u * (1.0 + g) + 2.0 * du * dg + u * d2g);
    } else {
        const double A = (upper || phi >= p.phi_T) ? p.Ap : p.Am;
        V = p.V0 + A * (phi - p.phi_T);
        dV = A;
        d2V = 0.0;
    }
}

}  // namespace fpt
