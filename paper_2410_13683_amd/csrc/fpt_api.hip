// fpt_api.hip -- the C ABI declared in include/fpt.h: argument validation,
// device memory of a context, launch configuration, histogram read-back, and
// the device kernel that evaluates the Bessel-ansatz noise table.
#include "fpt.h"
#include "internal.hpp"
#include "noise_node.hpp"
#include "potential.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <algorithm>
#include <vector>
#include <limits>
#include <mutex>

using namespace fpt;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    return fail(FPT_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(e_, #call); \
    } while (0)

bool is_finite(double v) { return std::isfinite(v); }

PotParams pot_params(const fpt_potential &p)
{
    return PotParams{p.kind, p.V0, p.phi_T, p.A_plus, p.A_minus, p.bump_m, p.bump_K, p.bump_Sigma};
}

double pot_V(const fpt_potential &p, double phi)
{
    double V, dV, d2V;
    pot_eval(pot_params(p), phi, false, V, dV, d2V);
    return V;
}

int check_potential(const fpt_potential *pot)
{
    if (!pot) return fail(FPT_EINVAL, "potential is NULL");
    if (pot->kind != FPT_POT_PIECEWISE_LINEAR && pot->kind != FPT_POT_EXPONENTIAL &&
        pot->kind != FPT_POT_GAUSSIAN_BUMP)
        return fail(FPT_EINVAL, "unknown potential kind %d", pot->kind);
    const double v[] = {pot->V0,      pot->phi_T,  pot->A_plus, pot->A_minus,  pot->phi_in,
                        pot->pi_in,   pot->phi_end, pot->bump_m, pot->bump_K, pot->bump_Sigma};
    for (double x : v)
        if (!is_finite(x)) return fail(FPT_EINVAL, "potential parameters must be finite");
    if (!(pot->V0 > 0.0)) return fail(FPT_EINVAL, "V0 must be > 0");
    if (pot->kind == FPT_POT_PIECEWISE_LINEAR && (pot->A_plus == 0.0 || pot->A_minus == 0.0))
        return fail(FPT_EINVAL, "A_plus and A_minus must be non-zero");
    if (pot->kind == FPT_POT_GAUSSIAN_BUMP &&
        (!(pot->bump_m > 0.0) || !(pot->bump_Sigma > 0.0) || !(pot->bump_K > -1.0)))
        return fail(FPT_EINVAL, "the Gaussian bump needs m > 0, Sigma > 0 and K > -1");
    return FPT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// noise table kernel: eq. (covariance_constant_nu) with eq. (nu_squared_approximation)
// ---------------------------------------------------------------------------
__global__ void table_bessel_kernel(PotParams pp, double sigma, int n, double phi_lo, double h, double *S,
                                    double *t, int *bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double phi = grid_node(phi_lo, j, h);
    double V, dV, d2V;
    pot_eval(pp, phi, false, V, dV, d2V);
    const double r1 = dV / V, r2 = d2V / V;   // V'/V, V''/V
    const double nu2 = 2.25 - 3.0 * (r2 - r1 * r1);
    if (!(V > 0.0) || !(nu2 > 0.0)) {
        atomicOr(bad, 1);
        S[j] = 0.0;
        t[j] = 0.0;
        return;
    }
    const double nu = sqrt(nu2);
    const double H = sqrt(V / 3.0);
    // sqrt(Xi_phiphi) = H/(2 pi) Gamma(nu)/Gamma(3/2) (sigma/2)^(3/2 - nu);  Gamma(3/2) = sqrt(pi)/2
    S[j] = H / (2.0 * M_PI) * (tgamma(nu) / (0.5 * sqrt(M_PI))) * pow(0.5 * sigma, 1.5 - nu);
    t[j] = nu - 1.5;   // Xi_phipi / Xi_phiphi
}

extern "C" int fpt_noise_table_bessel(const fpt_potential *pot, double sigma, int32_t n, double phi_lo,
                                      double phi_hi, double *S_out, double *tan_out)
{
    int rc = check_potential(pot);
    if (rc) return rc;
    if (n < 1 || n > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", n, FPT_MAX_TABLE);
    if (!(sigma > 0.0) || !is_finite(sigma)) return fail(FPT_EINVAL, "sigma must be finite and > 0");
    if (!is_finite(phi_lo) || !is_finite(phi_hi) || (n > 1 && !(phi_hi > phi_lo)))
        return fail(FPT_EINVAL, "need phi_hi > phi_lo");
    if (!S_out || !tan_out) return fail(FPT_EINVAL, "output arrays are NULL");
    const double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    double *d = nullptr;
    int *d_bad = nullptr;
    HIP_TRY(hipMalloc(&d, 2 * sizeof(double) * n + sizeof(int)));
    d_bad = reinterpret_cast<int *>(d + 2 * n);
    hipError_t e = hipMemset(d_bad, 0, sizeof(int));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(table_bessel_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, pot_params(*pot), sigma, n,
                           phi_lo, h, d, d + n, d_bad);
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpy(S_out, d, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(tan_out, d + n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "noise table kernel");
    if (bad) return fail(FPT_EINVAL, "V <= 0 or nu^2 <= 0 at a table node");
    return FPT_OK;
}

// ---------------------------------------------------------------------------
// 2D noise table kernel: eq. (covariance_matrix_direct) from the full
// Bunch-Davies mode of eq. (delta_phi_bessel) at -k eta = sigma
// ---------------------------------------------------------------------------
__global__ void table_bessel2d_kernel(PotParams pp, double sigma, int n, double phi_lo, double h, double *Xpp,
                                      double *Xpq, double *Xqq, int *bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (!bessel2d_node(pp, sigma, grid_node(phi_lo, j, h), Xpp[j], Xpq[j], Xqq[j])) atomicOr(bad, 1);
}

extern "C" int fpt_noise_table_bessel2d(const fpt_potential *pot, double sigma, int32_t n, double phi_lo,
                                        double phi_hi, double *Xpp_out, double *Xpq_out, double *Xqq_out)
{
    int rc = check_potential(pot);
    if (rc) return rc;
    if (n < 1 || n > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", n, FPT_MAX_TABLE);
    if (!(sigma > 0.0) || !(sigma <= 2.0)) return fail(FPT_EINVAL, "sigma must lie in (0, 2]");
    if (!is_finite(phi_lo) || !is_finite(phi_hi) || (n > 1 && !(phi_hi > phi_lo)))
        return fail(FPT_EINVAL, "need phi_hi > phi_lo");
    if (!Xpp_out || !Xpq_out || !Xqq_out) return fail(FPT_EINVAL, "output arrays are NULL");
    const double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    double *d = nullptr;
    HIP_TRY(hipMalloc(&d, 3 * sizeof(double) * n + sizeof(int)));
    int *d_bad = reinterpret_cast<int *>(d + 3 * n);
    hipError_t e = hipMemset(d_bad, 0, sizeof(int));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(table_bessel2d_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, pot_params(*pot), sigma, n,
                           phi_lo, h, d, d + n, d + 2 * n, d_bad);
        e = hipGetLastError();
    }
    int bad = 0;
    if (e == hipSuccess) e = hipMemcpy(Xpp_out, d, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Xpq_out, d + n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Xqq_out, d + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "2D noise table kernel");
    if (bad) return fail(FPT_EINVAL, "V <= 0, nu^2 <= 0 or nu near an integer at a table node");
    return FPT_OK;
}

// Bessel-matched table: trajectory and mode solves in fpt_table.hip.
extern "C" int fpt_noise_table_matched(const fpt_potential *pot, double sigma, int32_t n, double phi_lo,
                                       double phi_hi, double phi_start, double pi_start, double *S_out,
                                       double *tan_out, double *fac_out)
{
    int rc = check_potential(pot);
    if (rc) return rc;
    if (n < 1 || n > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", n, FPT_MAX_TABLE);
    if (!(sigma > 0.0) || !(sigma <= 2.0)) return fail(FPT_EINVAL, "sigma must lie in (0, 2]");
    if (!is_finite(phi_lo) || !is_finite(phi_hi) || (n > 1 && !(phi_hi > phi_lo)))
        return fail(FPT_EINVAL, "need phi_hi > phi_lo");
    if (!is_finite(phi_start) || !is_finite(pi_start)) return fail(FPT_EINVAL, "start must be finite");
    if (!(pot_V(*pot, phi_start) > 0.0)) return fail(FPT_EINVAL, "V(phi_start) must be > 0");
    if (!(0.5 * pi_start * pi_start < 1.0)) return fail(FPT_EINVAL, "the start needs eps1 = pi^2/2 < 1");
    if (!S_out || !tan_out) return fail(FPT_EINVAL, "output arrays are NULL");
    const double h = (n > 1) ? (phi_hi - phi_lo) / (double)(n - 1) : 0.0;
    const size_t scratch = fpt::matched_scratch_bytes(n);
    const size_t out_off = (scratch + 255) & ~(size_t)255;
    char *d = nullptr;
    HIP_TRY(hipMalloc(&d, out_off + 3 * sizeof(double) * n + sizeof(int)));
    double *d_S = reinterpret_cast<double *>(d + out_off);
    int *d_status = reinterpret_cast<int *>(d_S + 3 * n);
    hipError_t e = hipMemset(d_status, 0, sizeof(int));
    if (e == hipSuccess)
        e = fpt::matched_table_launch(pot_params(*pot), sigma, n, phi_lo, h, phi_start, pi_start, d, d_S, d_S + n,
                                      d_S + 2 * n, d_status, nullptr);
    int status = 0;
    if (e == hipSuccess) e = hipMemcpy(S_out, d_S, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(tan_out, d_S + n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && fac_out) e = hipMemcpy(fac_out, d_S + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&status, d_status, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "matched noise table kernels");
    if (status & 1) return fail(FPT_EINVAL, "V <= 0 or nu^2 <= 0 at a table node");
    if (status & 2) return fail(FPT_EINVAL, "a node is reached before its mode can start at k = 100 aH: start earlier");
    if (status & 4) return fail(FPT_EINVAL, "non-finite or zero Bessel coefficient at a node");
    return FPT_OK;
}

extern "C" int fpt_noise_table_matched_time(const fpt_potential *pot, double sigma, int32_t n, double t_lo,
                                            double t_hi, double phi_start, double pi_start, double phi_ref,
                                            double *S_out, double *tan_out, double *fac_out, double *phi_out)
{
    int rc = check_potential(pot);
    if (rc) return rc;
    if (n < 1 || n > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", n, FPT_MAX_TABLE);
    if (!(sigma > 0.0) || !(sigma <= 2.0)) return fail(FPT_EINVAL, "sigma must lie in (0, 2]");
    if (!is_finite(t_lo) || !is_finite(t_hi) || (n > 1 && !(t_hi > t_lo)))
        return fail(FPT_EINVAL, "need t_hi > t_lo");
    if (!is_finite(phi_start) || !is_finite(pi_start) || !is_finite(phi_ref))
        return fail(FPT_EINVAL, "start and phi_ref must be finite");
    if (!(phi_start > phi_ref)) return fail(FPT_EINVAL, "need phi_start > phi_ref");
    if (!(pot_V(*pot, phi_start) > 0.0)) return fail(FPT_EINVAL, "V(phi_start) must be > 0");
    if (!(0.5 * pi_start * pi_start < 1.0)) return fail(FPT_EINVAL, "the start needs eps1 = pi^2/2 < 1");
    if (!S_out || !tan_out) return fail(FPT_EINVAL, "output arrays are NULL");
    const double h = (n > 1) ? (t_hi - t_lo) / (double)(n - 1) : 0.0;
    const double N_after = (n > 1 ? t_hi : t_lo) + 2e-4;   // one sample beyond the last node
    const size_t out_off = (fpt::matched_time_scratch_bytes() + 255) & ~(size_t)255;
    char *d = nullptr;
    HIP_TRY(hipMalloc(&d, out_off + 4 * sizeof(double) * n + sizeof(int)));
    double *d_S = reinterpret_cast<double *>(d + out_off);
    int *d_status = reinterpret_cast<int *>(d_S + 4 * n);
    hipError_t e = hipMemset(d_status, 0, sizeof(int));
    if (e == hipSuccess)
        e = fpt::matched_time_launch(pot_params(*pot), sigma, n, t_lo, h, phi_start, pi_start, phi_ref, N_after, d,
                                     d_S, d_S + n, d_S + 2 * n, d_S + 3 * n, d_status, nullptr);
    int status = 0;
    if (e == hipSuccess) e = hipMemcpy(S_out, d_S, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(tan_out, d_S + n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && fac_out) e = hipMemcpy(fac_out, d_S + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && phi_out) e = hipMemcpy(phi_out, d_S + 3 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&status, d_status, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "time-node matched noise table kernels");
    if (status & 16)
        return fail(FPT_EINVAL, "the trajectory does not pass phi_ref, or a node lies outside the followed trajectory");
    if (status & 1) return fail(FPT_EINVAL, "V <= 0 or nu^2 <= 0 at a table node");
    if (status & 2) return fail(FPT_EINVAL, "a node is reached before its mode can start at k = 100 aH: start earlier");
    if (status & 4) return fail(FPT_EINVAL, "non-finite or zero Bessel coefficient at a node");
    return FPT_OK;
}

extern "C" int fpt_noise_table_bessel2d_time(const fpt_potential *pot, double sigma, int32_t n, double t_lo,
                                             double t_hi, double phi_start, double pi_start, double phi_ref,
                                             double *Xpp_out, double *Xpq_out, double *Xqq_out, double *phi_out)
{
    int rc = check_potential(pot);
    if (rc) return rc;
    if (n < 1 || n > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", n, FPT_MAX_TABLE);
    if (!(sigma > 0.0) || !(sigma <= 2.0)) return fail(FPT_EINVAL, "sigma must lie in (0, 2]");
    if (!is_finite(t_lo) || !is_finite(t_hi) || (n > 1 && !(t_hi > t_lo)))
        return fail(FPT_EINVAL, "need t_hi > t_lo");
    if (!is_finite(phi_start) || !is_finite(pi_start) || !is_finite(phi_ref))
        return fail(FPT_EINVAL, "start and phi_ref must be finite");
    if (!(phi_start > phi_ref)) return fail(FPT_EINVAL, "need phi_start > phi_ref");
    if (!(pot_V(*pot, phi_start) > 0.0)) return fail(FPT_EINVAL, "V(phi_start) must be > 0");
    if (!(0.5 * pi_start * pi_start < 1.0)) return fail(FPT_EINVAL, "the start needs eps1 = pi^2/2 < 1");
    if (!Xpp_out || !Xpq_out || !Xqq_out) return fail(FPT_EINVAL, "output arrays are NULL");
    const double h = (n > 1) ? (t_hi - t_lo) / (double)(n - 1) : 0.0;
    const double N_after = (n > 1 ? t_hi : t_lo) + 2e-4;   // one sample beyond the last node
    const size_t out_off = (fpt::matched_time_scratch_bytes() + 255) & ~(size_t)255;
    char *d = nullptr;
    HIP_TRY(hipMalloc(&d, out_off + 4 * sizeof(double) * n + sizeof(int)));
    double *d_X = reinterpret_cast<double *>(d + out_off);
    int *d_status = reinterpret_cast<int *>(d_X + 4 * n);
    hipError_t e = hipMemset(d_status, 0, sizeof(int));
    if (e == hipSuccess)
        e = fpt::bessel2d_time_launch(pot_params(*pot), sigma, n, t_lo, h, phi_start, pi_start, phi_ref, N_after, d,
                                      d_X, d_X + n, d_X + 2 * n, d_X + 3 * n, d_status, nullptr);
    int status = 0;
    if (e == hipSuccess) e = hipMemcpy(Xpp_out, d_X, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Xpq_out, d_X + n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(Xqq_out, d_X + 2 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && phi_out) e = hipMemcpy(phi_out, d_X + 3 * n, sizeof(double) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&status, d_status, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(e, "time-node 2D noise table kernels");
    if (status & 16)
        return fail(FPT_EINVAL, "the trajectory does not pass phi_ref, or a node lies outside the followed trajectory");
    if (status & 1) return fail(FPT_EINVAL, "V <= 0, nu^2 <= 0 or nu near an integer at a table node");
    return FPT_OK;
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct fpt_ctx {
    int device = 0;
    int cu_count = 0;
    size_t lds_per_block_max = 0;
    int precision = FPT_FP64;
    fpt_options opt{};
    Inst inst{};
    unsigned long long *cursor = nullptr;
    void *d_mem = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_done = nullptr;
    bool ran = false;                        // ev_start/ev_stop bracket the last fpt_run's kernel
    bool pending = false;                    // ev_done marks the end of the last work on the accumulators
    hipStream_t io_stream = nullptr;         // the context's own stream for reading and clearing them
    uint64_t n_traj_total = 0;
    bool drift_table_used = false;           // FP32 V'/V intervals (see build_drift_table)
    // learned control (FPT_BIAS_MLP)
    GridSpec grid{};
    void *d_mlp = nullptr;                   // fixed-size part, carved below
    float *d_params = nullptr, *d_adam_m = nullptr, *d_adam_v = nullptr;
    double *d_node_a = nullptr, *d_G = nullptr, *d_work = nullptr, *d_J = nullptr;
    double2 *d_grid64 = nullptr;
    float4 *d_grid32 = nullptr;
    unsigned long long *d_counters = nullptr;  // [0] tail count of a slice, [1] total, [2] mismatches, [3] replay cursor
    void *d_train_acc = nullptr;             // private histogram of gradient runs
    int adam_t = 0;
    // per-trajectory scratch of gradient runs, grown on demand
    void *d_scratch = nullptr;
    size_t scratch_cap = 0;
};

static const size_t kGradSlice = size_t(1) << 22;

// Symmetric positive semi-definite square root of [[a, b], [b, c]]:
// (Xi + sqrt(det) 1)/sqrt(tr + 2 sqrt(det)) (Cayley-Hamilton); zero for Xi = 0.
static void sym_sqrt2(double a, double b, double c, double &Spp, double &Spq, double &Sqq)
{
    const double s = std::sqrt(std::max(a * c - b * b, 0.0));
    const double t2 = a + c + 2.0 * s;
    if (t2 == 0.0) {
        Spp = Spq = Sqq = 0.0;
        return;
    }
    const double t = std::sqrt(t2);
    Spp = (a + s) / t;
    Spq = b / t;
    Sqq = (c + s) / t;
}

// Unit eigenvector of [[a, b], [b, c]] for its largest eigenvalue, phi component >= 0;
// (1, 0) when the eigenvalues coincide or the matrix is zero.
static void principal_axis2(double a, double b, double c, double &e1, double &e2)
{
    const double r = std::sqrt(0.25 * (a - c) * (a - c) + b * b);
    double v1 = a >= c ? 0.5 * (a - c) + r : b;
    double v2 = a >= c ? b : 0.5 * (c - a) + r;
    if (v1 < 0.0) {
        v1 = -v1;
        v2 = -v2;
    }
    const double nrm = std::sqrt(v1 * v1 + v2 * v2);
    if (nrm == 0.0) {
        e1 = 1.0;
        e2 = 0.0;
        return;
    }
    e1 = v1 / nrm;
    e2 = v2 / nrm;
}

// V'/V per interval of the noise table for the FP32-state kernels: entry j is
// (r(phi_j), r(phi_j+1) - r(phi_j)) on the potential branch of interval j, with
// r = V'/V, so r is the linear interpolation of the interval.  The branch kink
// phi_T must be a node (or lie outside the table) and the interpolation must
// stay within 2^-25 of V'/V at every interval's midpoint; otherwise every entry
// is NaN.  The entries of the two edge intervals (where coordinates outside the
// table are clamped) and of the two intervals that meet at phi_T (where the
// FP32 coordinate may round to the wrong side) are always NaN.  The kernels
// compute V'/V exactly wherever they read NaN.  Returns whether any entry is
// usable.
static bool build_drift_table(const fpt_potential &p, int nt, double phi_lo, double phi_hi, std::vector<float> &r)
{
    const float nan = std::numeric_limits<float>::quiet_NaN();
    r.assign(2 * (size_t)nt, nan);
    if (nt < 4) return false;
    const double h = (phi_hi - phi_lo) / (double)(nt - 1);
    int j_T = -1;                             // node at the kink, if inside the table
    if (p.kind == FPT_POT_PIECEWISE_LINEAR && p.phi_T > phi_lo && p.phi_T < phi_hi) {
        const double q = (p.phi_T - phi_lo) / h;
        const double qr = std::nearbyint(q);
        if (std::fabs(q - qr) > 1e-9) return false;
        j_T = (int)qr;
    }
    std::vector<float> t(2 * (size_t)nt, nan);
    for (int j = 0; j + 1 < nt; ++j) {
        const double a = phi_lo + (double)j * h, b = phi_lo + (double)(j + 1) * h, m = 0.5 * (a + b);
        double ra, rb, rm;
        if (p.kind == FPT_POT_EXPONENTIAL) {
            ra = rb = rm = p.A_plus;
        } else {
            const double A = (m >= p.phi_T) ? p.A_plus : p.A_minus;
            const double Va = p.V0 + A * (a - p.phi_T), Vb = p.V0 + A * (b - p.phi_T), Vm = p.V0 + A * (m - p.phi_T);
            if (!(Va > 0.0 && Vb > 0.0 && Vm > 0.0)) return false;
            ra = A / Va;
            rb = A / Vb;
            rm = A / Vm;
        }
        if (!(std::fabs(0.5 * (ra + rb) - rm) <= 0x1p-25 * std::fabs(rm))) return false;
        t[2 * j] = (float)ra;
        t[2 * j + 1] = (float)(rb - ra);
    }
    auto mark = [&](int j) {
        if (j >= 0 && j + 1 < nt) t[2 * j] = t[2 * j + 1] = nan;
    };
    mark(0);
    mark(nt - 2);
    if (j_T >= 0) {
        mark(j_T - 1);
        mark(j_T);
    }
    r = t;
    return true;
}

// Device memory and first tabulation of the learned control of context c
// (bias already validated).  Grid coordinates of the kernels:
//   u0 = (x0 - lo0)(n0 - 1)/(hi0 - lo0) with x0 = (phi - c0)/s0, i.e. phi k0 + off0,
//   u1 likewise from ln max(|pi|, 1e-30).
static int mlp_setup(fpt_ctx *c, const fpt_bias &b)
{
    GridSpec &g = c->grid;
    g.n0 = b.grid_n[0];
    g.n1 = b.grid_n[1];
    g.lo0 = b.grid_range[0];
    g.hi0 = b.grid_range[1];
    g.lo1 = b.grid_range[2];
    g.hi1 = b.grid_range[3];
    const size_t nn = (size_t)g.n0 * g.n1, nc = (size_t)(g.n0 - 1) * (g.n1 - 1);
    const size_t nbytes_p = sizeof(float) * FPT_MLP_NPARAM;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off = (off + bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t o_params = carve(nbytes_p), o_m = carve(2 * nbytes_p);   // m and v adjacent
    const size_t o_node = carve(8 * nn), o_G = carve(8 * nn), o_work = carve(8 * 4 * nn * kMlpHidden);
    const size_t o_J = carve(8), o_g64 = carve(32 * nc), o_g32 = carve(16 * nc), o_cnt = carve(8 * 4);
    const size_t o_acc = carve(acc_bytes(c->opt.n_bins));
    HIP_TRY(hipMalloc(&c->d_mlp, off));
    unsigned char *base = static_cast<unsigned char *>(c->d_mlp);
    c->d_params = reinterpret_cast<float *>(base + o_params);
    c->d_adam_m = reinterpret_cast<float *>(base + o_m);
    c->d_adam_v = c->d_adam_m + FPT_MLP_NPARAM;
    c->d_node_a = reinterpret_cast<double *>(base + o_node);
    c->d_G = reinterpret_cast<double *>(base + o_G);
    c->d_work = reinterpret_cast<double *>(base + o_work);
    c->d_J = reinterpret_cast<double *>(base + o_J);
    c->d_grid64 = reinterpret_cast<double2 *>(base + o_g64);
    c->d_grid32 = reinterpret_cast<float4 *>(base + o_g32);
    c->d_counters = reinterpret_cast<unsigned long long *>(base + o_cnt);
    c->d_train_acc = base + o_acc;
    HIP_TRY(hipMemset(c->d_mlp, 0, off));
    HIP_TRY(hipMemcpy(c->d_params, b.mlp_params, nbytes_p, hipMemcpyHostToDevice));
    Inst &I = c->inst;
    I.bias_kind = kBiasMlp;
    I.g_n0 = g.n0;
    I.g_n1 = g.n1;
    const double q0 = (double)(g.n0 - 1) / (g.hi0 - g.lo0), q1 = (double)(g.n1 - 1) / (g.hi1 - g.lo1);
    I.g_k0 = q0 / b.norm[1];
    I.g_off0 = -(b.norm[0] / b.norm[1] + g.lo0) * q0;
    I.g_k1 = q1 / b.norm[3];
    I.g_off1 = -(b.norm[2] / b.norm[3] + g.lo1) * q1;
    I.grid64 = c->d_grid64;
    I.grid32 = c->d_grid32;
    I.mlp_every = b.mlp_every;
    I.mlp_params = c->d_params;
    I.m_k0 = 1.0 / b.norm[1];
    I.m_off0 = -b.norm[0] / b.norm[1];
    I.m_k1 = 1.0 / b.norm[3];
    I.m_off1 = -b.norm[2] / b.norm[3];
    HIP_TRY(mlp_tabulate(c->d_params, g, c->d_node_a, c->d_grid64, c->d_grid32, nullptr));
    HIP_TRY(hipDeviceSynchronize());
    return FPT_OK;
}

extern "C" int fpt_create(const fpt_potential *pot, const fpt_noise_table *table, const fpt_bias *bias,
                          const fpt_options *opts, fpt_ctx **out)
{
    if (!out) return fail(FPT_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = check_potential(pot);
    if (rc) return rc;
    if (!table || !opts) return fail(FPT_EINVAL, "table or options is NULL");
    if (!(pot->phi_in > pot->phi_end)) return fail(FPT_EINVAL, "need phi_in > phi_end");
    if (pot->kind == FPT_POT_PIECEWISE_LINEAR) {
        // V is linear on each side of phi_T: its minimum on [phi_end, phi_in] is at an end or at phi_T
        bool ok = pot_V(*pot, pot->phi_end) > 0.0 && pot_V(*pot, pot->phi_in) > 0.0;
        if (pot->phi_T > pot->phi_end && pot->phi_T < pot->phi_in) ok = ok && pot_V(*pot, pot->phi_T) > 0.0;
        if (!ok) return fail(FPT_EINVAL, "V <= 0 on [phi_end, phi_in]");
    }
    if (pot->kind == FPT_POT_GAUSSIAN_BUMP) {
        // V > 0 wherever phi != 0 (m > 0, K > -1); the run stays at phi > phi_end
        if (!(pot->phi_end > 0.0)) return fail(FPT_EINVAL, "the Gaussian bump needs phi_end > 0");
        if (opts && opts->precision != FPT_FP64)
            return fail(FPT_EUNSUPPORTED, "the Gaussian bump is implemented with FP64 state only");
        if (bias && bias->kind == FPT_BIAS_MLP)
            return fail(FPT_EUNSUPPORTED, "the Gaussian bump takes no learned bias");
        if (table && table->dim == 2) return fail(FPT_EUNSUPPORTED, "the Gaussian bump takes 1D noise only");
    }
    // noise table
    const int nt = table->n;
    if (nt < 1 || nt > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", nt, FPT_MAX_TABLE);
    const int dim = table->dim == 2 ? 2 : 1;
    if (table->dim != 0 && table->dim != 1 && table->dim != 2) return fail(FPT_EINVAL, "table dim must be 1 or 2");
    if (table->axis != FPT_AXIS_PHI && table->axis != FPT_AXIS_TIME)
        return fail(FPT_EINVAL, "table axis must be FPT_AXIS_PHI or FPT_AXIS_TIME");
    const bool time_axis = table->axis == FPT_AXIS_TIME && nt > 1;
    if (time_axis && bias && bias->kind == FPT_BIAS_MLP)
        return fail(FPT_EUNSUPPORTED, "a time-indexed table takes no learned bias");
    if (dim == 1) {
        if (!table->S || !table->tan_theta) return fail(FPT_EINVAL, "table arrays are NULL");
        for (int i = 0; i < nt; ++i) {
            if (!is_finite(table->S[i]) || !is_finite(table->tan_theta[i]))
                return fail(FPT_EINVAL, "table entries must be finite");
            if (table->S[i] < 0.0) return fail(FPT_EINVAL, "table S must be >= 0");
        }
    } else {
        if (!table->Xi_pp || !table->Xi_pq || !table->Xi_qq) return fail(FPT_EINVAL, "2D table arrays are NULL");
        for (int i = 0; i < nt; ++i) {
            const double a = table->Xi_pp[i], b = table->Xi_pq[i], c = table->Xi_qq[i];
            if (!is_finite(a) || !is_finite(b) || !is_finite(c)) return fail(FPT_EINVAL, "table entries must be finite");
            const bool zero = a == 0.0 && b == 0.0 && c == 0.0;
            if (!zero && !(a > 0.0 && a * c - b * b > 0.0))
                return fail(FPT_EINVAL, "2D table node %d is neither zero nor positive definite", i);
        }
        if (bias && bias->kind == FPT_BIAS_MLP) return fail(FPT_EUNSUPPORTED, "2D noise takes no learned bias");
    }
    if (nt > 1 && (!is_finite(table->phi_lo) || !is_finite(table->phi_hi) || !(table->phi_hi > table->phi_lo)))
        return fail(FPT_EINVAL, "table needs phi_hi > phi_lo");
    // bias
    fpt_bias b{};
    if (bias) b = *bias;
    if (b.kind != FPT_BIAS_NONE && b.kind != FPT_BIAS_CONST && b.kind != FPT_BIAS_MLP)
        return fail(FPT_EINVAL, "unknown bias kind %d", b.kind);
    if (!is_finite(b.A)) return fail(FPT_EINVAL, "bias amplitude must be finite");
    if (b.kind == FPT_BIAS_MLP) {
        if (!b.mlp_params) return fail(FPT_EINVAL, "MLP bias needs mlp_params");
        for (int i = 0; i < 4; ++i)
            if (!is_finite(b.norm[i]) || !is_finite(b.grid_range[i])) return fail(FPT_EINVAL, "MLP norm and grid range must be finite");
        if (b.norm[1] == 0.0 || b.norm[3] == 0.0) return fail(FPT_EINVAL, "MLP norm scales must be non-zero");
        if (b.mlp_every < 0) return fail(FPT_EINVAL, "mlp_every must be >= 0");
        if (b.grid_n[0] < 2 || b.grid_n[1] < 2 || (int64_t)b.grid_n[0] * b.grid_n[1] > FPT_MLP_MAX_GRID)
            return fail(FPT_EINVAL, "MLP grid needs 2 <= n0, n1 and n0 n1 <= %d", FPT_MLP_MAX_GRID);
        if (!(b.grid_range[1] > b.grid_range[0]) || !(b.grid_range[3] > b.grid_range[2]))
            return fail(FPT_EINVAL, "MLP grid ranges need hi > lo");
        for (int i = 0; i < FPT_MLP_NPARAM; ++i)
            if (!std::isfinite(b.mlp_params[i])) return fail(FPT_EINVAL, "MLP parameters must be finite");
    }
    // options
    const fpt_options &o = *opts;
    if (o.precision != FPT_FP64 && o.precision != FPT_FP32_STATE)
        return fail(FPT_EINVAL, "unknown precision %d", o.precision);
    if (o.n_bins < 1 || o.n_bins > FPT_MAX_BINS) return fail(FPT_EINVAL, "n_bins out of 1..%d", FPT_MAX_BINS);
    if (!is_finite(o.lo) || !is_finite(o.hi) || !is_finite(o.N_ref) || !(o.hi > o.lo))
        return fail(FPT_EINVAL, "histogram needs finite lo < hi and N_ref");
    if (o.bins_kind == FPT_BINS_LOG) {
        if (!(o.lo > 0.0)) return fail(FPT_EINVAL, "log bins need lo > 0");
    } else if (o.bins_kind != FPT_BINS_LINEAR) {
        return fail(FPT_EINVAL, "unknown bins kind %d", o.bins_kind);
    }
    if (o.max_steps < 1 || o.max_steps > FPT_MAX_STEPS) return fail(FPT_EINVAL, "max_steps out of 1..2^30-1");
    if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 1024 || o.block_size % 64))
        return fail(FPT_EINVAL, "block_size must be a multiple of 64 in 64..1024");
    if (o.blocks_per_cu < 0) return fail(FPT_EINVAL, "blocks_per_cu must be >= 0");
    if (o.chunk != 0 && (o.chunk < 4 || o.chunk % 4)) return fail(FPT_EINVAL, "chunk must be a positive multiple of 4");

    fpt_ctx *c = new (std::nothrow) fpt_ctx();
    if (!c) return fail(FPT_ENOMEM, "host allocation failed");
    c->opt = o;
    c->precision = o.precision;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device);
    int lds_max = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    c->lds_per_block_max = (size_t)lds_max;
    // device memory: FP64 table (nt x double2), FP32 table (nt x float4), FP32 V'/V intervals
    // (nt x float2), cursor, accumulators
    const size_t off_tab32 = sizeof(double) * 2 * nt;
    const size_t off_rtab = off_tab32 + sizeof(float) * 4 * nt;
    const size_t off_tab2d = (off_rtab + sizeof(float) * 2 * nt + 15) & ~size_t(15);
    const size_t off_tab2d32 = off_tab2d + (dim == 2 ? sizeof(double) * 6 * nt : 0);
    const size_t off_cursor = (off_tab2d32 + (dim == 2 ? sizeof(float) * 12 * nt : 0) + 255) & ~size_t(255);
    const size_t off_acc = off_cursor + 256;
    const size_t total = off_acc + acc_bytes(o.n_bins);
    if (e == hipSuccess) e = hipMalloc(&c->d_mem, total);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "fpt_create device setup");
    }
    std::vector<double> h64(2 * nt);
    std::vector<float> h32(4 * nt);
    bool all_pos = true;
    std::vector<double> h2d(dim == 2 ? 6 * (size_t)nt : 0);
    for (int i = 0; i < nt && dim == 1; ++i) {
        const int k = (i + 1 < nt) ? i + 1 : i;
        h64[2 * i] = table->S[i];
        h64[2 * i + 1] = table->tan_theta[i];
        const float S = (float)table->S[i], St = (float)table->tan_theta[i];
        h32[4 * i] = S;
        h32[4 * i + 1] = (float)table->S[k] - S;
        h32[4 * i + 2] = St;
        h32[4 * i + 3] = (float)table->tan_theta[k] - St;
        all_pos = all_pos && table->S[i] > 0.0;
    }
    for (int i = 0; i < nt && dim == 2; ++i) {
        const double a = table->Xi_pp[i], b = table->Xi_pq[i], cc = table->Xi_qq[i];
        double *q = &h2d[6 * (size_t)i];
        sym_sqrt2(a, b, cc, q[0], q[1], q[2]);
        principal_axis2(a, b, cc, q[3], q[4]);
        q[5] = 0.0;
        all_pos = all_pos && !(a == 0.0 && b == 0.0 && cc == 0.0);
    }
    unsigned char *base = static_cast<unsigned char *>(c->d_mem);
    e = hipMemcpy(base, h64.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + off_tab32, h32.data(), sizeof(float) * 4 * nt, hipMemcpyHostToDevice);
    std::vector<float> hr;
    // the V'/V intervals follow phi nodes: a time-indexed table leaves them all NaN (computed exactly)
    if (time_axis) hr.assign(2 * (size_t)nt, std::numeric_limits<float>::quiet_NaN());
    else c->drift_table_used = build_drift_table(*pot, nt, table->phi_lo, table->phi_hi, hr);
    if (e == hipSuccess) e = hipMemcpy(base + off_rtab, hr.data(), sizeof(float) * 2 * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess && dim == 2)
        e = hipMemcpy(base + off_tab2d, h2d.data(), sizeof(double) * h2d.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && dim == 2) {
        // FP32 records: value and slope to the next node of S_pp, S_pq, S_qq, e_phi, e_pi (the last
        // node's slopes 0), then the V'/V interval of the FP32 table
        std::vector<float> h2f(12 * (size_t)nt);
        for (int i = 0; i < nt; ++i) {
            const int k = (i + 1 < nt) ? i + 1 : i;
            const double *q = &h2d[6 * (size_t)i], *qk = &h2d[6 * (size_t)k];
            float *f = &h2f[12 * (size_t)i];
            for (int m = 0; m < 5; ++m) {
                f[2 * m] = (float)q[m];
                f[2 * m + 1] = (float)qk[m] - (float)q[m];
            }
            f[10] = hr[2 * (size_t)i];
            f[11] = hr[2 * (size_t)i + 1];
        }
        e = hipMemcpy(base + off_tab2d32, h2f.data(), sizeof(float) * h2f.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(base + off_cursor, 0, 256 + acc_bytes(o.n_bins));
    if (e == hipSuccess) e = hipEventCreate(&c->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_stop);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->io_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        fpt_destroy(c);
        return hip_fail(e, "fpt_create initialisation");
    }
    Inst &I = c->inst;
    I.pot_kind = pot->kind;
    I.V0 = pot->V0; I.phi_T = pot->phi_T; I.A_plus = pot->A_plus; I.A_minus = pot->A_minus;
    I.phi_in = pot->phi_in; I.pi_in = pot->pi_in; I.phi_end = pot->phi_end;
    I.bump_m2 = pot->bump_m * pot->bump_m; I.bump_K = pot->bump_K; I.bump_Sigma = pot->bump_Sigma;
    I.n_tab = nt;
    I.tab_axis = time_axis ? 1 : 0;
    I.phi_lo = (nt > 1) ? table->phi_lo : 0.0;
    I.inv_h = (nt > 1) ? (double)(nt - 1) / (table->phi_hi - table->phi_lo) : 0.0;
    I.tab64 = reinterpret_cast<const double2 *>(base);
    I.tab32 = reinterpret_cast<const float4 *>(base + off_tab32);
    I.rtab32 = reinterpret_cast<const float2 *>(base + off_rtab);
    I.rec_S = I.rec_dS = I.rec_t = I.rec_dt = I.rec_r = I.rec_dr = 0.0f;
    for (int i = 0; i < nt && dim == 1; ++i) {
        if (!(hr[2 * (size_t)i] == hr[2 * (size_t)i])) continue;      // NaN-marked: read per step
        I.rec_S = std::max(I.rec_S, std::fabs(h32[4 * (size_t)i]));
        I.rec_dS = std::max(I.rec_dS, std::fabs(h32[4 * (size_t)i + 1]));
        I.rec_t = std::max(I.rec_t, std::fabs(h32[4 * (size_t)i + 2]));
        I.rec_dt = std::max(I.rec_dt, std::fabs(h32[4 * (size_t)i + 3]));
        I.rec_r = std::max(I.rec_r, std::fabs(hr[2 * (size_t)i]));
        I.rec_dr = std::max(I.rec_dr, std::fabs(hr[2 * (size_t)i + 1]));
    }
    I.noise_dim = dim;
    I.tab64_2d = reinterpret_cast<const double2 *>(base + off_tab2d);
    I.tab32_2d = reinterpret_cast<const float4 *>(base + off_tab2d32);
    I.all_S_pos = all_pos ? 1 : 0;
    I.bias_kind = b.kind;
    I.A = (b.kind == FPT_BIAS_CONST) ? b.A : 0.0;
    I.instance = o.instance;
    I.max_steps = (uint32_t)o.max_steps;
    I.hist.bins_kind = o.bins_kind;
    I.hist.n_bins = o.n_bins;
    I.hist.lo = o.lo;
    I.hist.N_ref = o.N_ref;
    I.hist.scale = (o.bins_kind == FPT_BINS_LINEAR) ? (double)o.n_bins / (o.hi - o.lo)
                                                    : (double)o.n_bins / std::log(o.hi / o.lo);
    I.acc = base + off_acc;
    c->cursor = reinterpret_cast<unsigned long long *>(base + off_cursor);
    if (b.kind == FPT_BIAS_MLP) {
        rc = mlp_setup(c, b);
        if (rc) {
            fpt_destroy(c);
            return rc;
        }
    }
    const int n_cells = grid_cells(I);
    size_t need = dim == 2 ? em2d_lds_bytes(o.n_bins, nt, o.precision)
                           : em_lds_bytes(o.n_bins, nt, o.precision, n_cells, b.kind == FPT_BIAS_MLP && b.mlp_every > 0);
    if (b.kind == FPT_BIAS_MLP)
        need = std::max(need, replay_lds_bytes(nt, o.precision, n_cells, c->grid.n0 * c->grid.n1));
    if (need > c->lds_per_block_max) {
        fpt_destroy(c);
        return fail(FPT_EINVAL, "noise table, control grid and histogram do not fit in LDS (%zu > %zu bytes)", need,
                    (size_t)lds_max);
    }
    *out = c;
    return FPT_OK;
}

static int occupancy_grid(const void *fn, int block, size_t lds, int cu_count, int per_cu, int &grid)
{
    if (per_cu == 0) {
        int occ = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fn, block, lds);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        per_cu = occ > 0 ? occ : 1;
    }
    grid = per_cu * cu_count;
    if (grid < 1) grid = 1;
    return FPT_OK;
}

extern "C" int fpt_run(fpt_ctx *c, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                       void *hip_stream, double *d_N, double *d_lnw, uint32_t *d_steps)
{
    if (!c) return fail(FPT_EINVAL, "context is NULL");
    if (!(dN > 0.0) || !is_finite(dN)) return fail(FPT_EINVAL, "dN must be finite and > 0");
    if (traj_offset + n_traj < traj_offset) return fail(FPT_EINVAL, "trajectory range overflows 64 bits");
    if (n_traj == 0) return FPT_OK;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(FPT_ESTATE, "current device %d differs from the context's %d", dev, c->device);
    EmParams p{};
    p.inst = c->inst;
    p.run.dN = dN;
    p.run.sqrt_dN = std::sqrt(dN);
    p.run.key0 = (uint32_t)seed;
    p.run.key1 = (uint32_t)(seed >> 32);
    p.run.chunk = c->opt.chunk ? c->opt.chunk : 128;
    p.traj_offset = traj_offset;
    p.n_traj = n_traj;
    p.d_N = d_N;
    p.d_lnw = d_lnw;
    p.d_steps = d_steps;
    p.cursor = c->cursor;
    const int block = c->opt.block_size ? c->opt.block_size : 1024;
    int grid = 0;
    const bool two_d = c->inst.noise_dim == 2;
    // the learned control runs its tabulated network, or the network itself every mlp_every steps
    const bool exact = c->inst.bias_kind == kBiasMlp && c->inst.mlp_every > 0;
    const int bias_k = exact ? kBiasMlpExact : c->inst.bias_kind;
    const void *fn = two_d ? em2d_kernel_ptr(c->precision, c->inst.bias_kind, c->inst.all_S_pos != 0,
                                             tab_mode(c->inst) == 2)
                           : em_kernel_ptr(c->precision, bias_k, tab_mode(c->inst), c->inst.all_S_pos != 0,
                                           c->inst.pot_kind);
    const size_t lds = two_d ? em2d_lds_bytes(c->inst.hist.n_bins, c->inst.n_tab, c->precision)
                             : em_lds_bytes(c->inst.hist.n_bins, c->inst.n_tab, c->precision, grid_cells(c->inst),
                                            exact);
    int rc = occupancy_grid(fn, block, lds, c->cu_count, c->opt.blocks_per_cu, grid);
    if (rc) return rc;
    HIP_TRY(zero_words(p.cursor, 1, s));
    HIP_TRY(hipEventRecord(c->ev_start, s));
    if (two_d) HIP_TRY(em2d_launch(p, c->precision, grid, block, s));
    else HIP_TRY(em_launch(p, c->precision, grid, block, s, exact));
    HIP_TRY(hipEventRecord(c->ev_stop, s));
    HIP_TRY(hipEventRecord(c->ev_done, s));
    c->ran = true;
    c->pending = true;
    c->n_traj_total += n_traj;
    return FPT_OK;
}

extern "C" int fpt_last_kernel_ms(fpt_ctx *c, double *ms)
{
    if (!c || !ms) return fail(FPT_EINVAL, "NULL argument");
    if (!c->ran) return fail(FPT_ESTATE, "no run recorded");
    HIP_TRY(hipEventSynchronize(c->ev_stop));
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, c->ev_start, c->ev_stop));
    *ms = (double)f;
    return FPT_OK;
}

// Order the context's own stream after the last work recorded on its accumulators (its event:
// other streams and contexts on the device are not waited for).
static int wait_context(fpt_ctx *c)
{
    if (c->pending) HIP_TRY(hipStreamWaitEvent(c->io_stream, c->ev_done, 0));
    return FPT_OK;
}

static int read_acc(const void *d_acc, int n_bins, fpt_hist *out, uint64_t n_traj_total, hipStream_t s)
{
    const int nb = n_bins + 2;
    std::vector<unsigned char> h(acc_bytes(n_bins));
    HIP_TRY(hipMemcpyAsync(h.data(), d_acc, h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const unsigned long long *cnt = reinterpret_cast<const unsigned long long *>(h.data());
    const double *sum = reinterpret_cast<const double *>(cnt + nb + 4);
    for (int i = 0; i < nb; ++i) {
        out->count[i] = cnt[i];
        out->sum_w_bin[i] = sum[i];
        out->sum_w2_bin[i] = sum[nb + i];
        out->sum_lnw_bin[i] = sum[2 * nb + i];
        out->sum_lnw2_bin[i] = sum[3 * nb + i];
    }
    out->n_traj = n_traj_total;
    out->n_censored = cnt[nb + 0];
    out->n_ended_early = cnt[nb + 1];
    out->n_steps_total = cnt[nb + 2];
    out->sum_w = sum[4 * nb + 0];
    out->sum_w2 = sum[4 * nb + 1];
    out->sum_wN = sum[4 * nb + 2];
    out->sum_wN2 = sum[4 * nb + 3];
    return FPT_OK;
}

extern "C" int fpt_histogram(fpt_ctx *c, fpt_hist *out)
{
    if (!c || !out) return fail(FPT_EINVAL, "NULL argument");
    if (!out->count || !out->sum_w_bin || !out->sum_w2_bin || !out->sum_lnw_bin || !out->sum_lnw2_bin)
        return fail(FPT_EINVAL, "histogram arrays are NULL");
    int rc = wait_context(c);
    if (rc) return rc;
    return read_acc(c->inst.acc, c->opt.n_bins, out, c->n_traj_total, c->io_stream);
}

extern "C" int fpt_reset(fpt_ctx *c)
{
    if (!c) return fail(FPT_EINVAL, "context is NULL");
    int rc = wait_context(c);
    if (rc) return rc;
    // cleared by a kernel on the context's own stream after its last work, then waited for
    HIP_TRY(zero_words(reinterpret_cast<unsigned long long *>(c->inst.acc), acc_words(c->opt.n_bins), c->io_stream));
    HIP_TRY(hipStreamSynchronize(c->io_stream));
    c->pending = false;
    c->n_traj_total = 0;
    return FPT_OK;
}

extern "C" void fpt_destroy(fpt_ctx *c)
{
    if (!c) return;
    // teardown errors cannot be reported through a void function
    (void)hipDeviceSynchronize();
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    if (c->io_stream) (void)hipStreamDestroy(c->io_stream);
    if (c->d_mem) (void)hipFree(c->d_mem);
    if (c->d_mlp) (void)hipFree(c->d_mlp);
    if (c->d_scratch) (void)hipFree(c->d_scratch);
    delete c;
}

// ---------------------------------------------------------------------------
// learned control: parameters, gradient, Adam
// ---------------------------------------------------------------------------
static int mlp_check(fpt_ctx *c)
{
    if (!c) return fail(FPT_EINVAL, "context is NULL");
    if (c->inst.bias_kind != kBiasMlp) return fail(FPT_EINVAL, "the context has no learned bias");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != c->device) return fail(FPT_ESTATE, "current device %d differs from the context's %d", dev, c->device);
    return FPT_OK;
}

extern "C" int fpt_mlp_set(fpt_ctx *c, const float *params, void *hip_stream)
{
    int rc = mlp_check(c);
    if (rc) return rc;
    if (!params) return fail(FPT_EINVAL, "params is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(c->d_params, params, sizeof(float) * FPT_MLP_NPARAM, hipMemcpyDefault, s));
    // the Adam moments m and v are adjacent: 2 x 4482 floats = 4482 words
    HIP_TRY(zero_words(reinterpret_cast<unsigned long long *>(c->d_adam_m), FPT_MLP_NPARAM, s));
    c->adam_t = 0;
    HIP_TRY(mlp_tabulate(c->d_params, c->grid, c->d_node_a, c->d_grid64, c->d_grid32, s));
    return FPT_OK;
}

extern "C" int fpt_mlp_get(fpt_ctx *c, float *params, void *hip_stream)
{
    int rc = mlp_check(c);
    if (rc) return rc;
    if (!params) return fail(FPT_EINVAL, "params is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    HIP_TRY(hipMemcpyAsync(params, c->d_params, sizeof(float) * FPT_MLP_NPARAM, hipMemcpyDefault, s));
    HIP_TRY(hipStreamSynchronize(s));
    return FPT_OK;
}

extern "C" int fpt_mlp_table(fpt_ctx *c, double *a_out)
{
    int rc = mlp_check(c);
    if (rc) return rc;
    if (!a_out) return fail(FPT_EINVAL, "a_out is NULL");
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(a_out, c->d_node_a, sizeof(double) * c->grid.n0 * c->grid.n1, hipMemcpyDeviceToHost));
    return FPT_OK;
}

// Argument checks shared by the two gradient entry points.
static int mlp_grad_check(fpt_ctx *c, uint64_t n_traj, double dN, uint64_t traj_offset, double tail_lo,
                          int32_t objective, const float *d_grad)
{
    int rc = mlp_check(c);
    if (rc) return rc;
    if (c->inst.mlp_every > 0)
        return fail(FPT_EUNSUPPORTED, "the replay gradient is that of the tabulated network (mlp_every = 0)");
    if (!d_grad) return fail(FPT_EINVAL, "d_grad is NULL");
    if (!(dN > 0.0) || !is_finite(dN)) return fail(FPT_EINVAL, "dN must be finite and > 0");
    if (!is_finite(tail_lo)) return fail(FPT_EINVAL, "tail_lo must be finite");
    if (objective != FPT_MLP_OBJ_J && objective != FPT_MLP_OBJ_LOG_J)
        return fail(FPT_EINVAL, "unknown objective %d", objective);
    if (n_traj == 0) return fail(FPT_EINVAL, "n_traj must be > 0");
    if (traj_offset + n_traj < traj_offset) return fail(FPT_EINVAL, "trajectory range overflows 64 bits");
    return FPT_OK;
}

// The gradient run of fpt_mlp_grad on per-trajectory scratch sb of cap trajectories (N, ln w, steps
// and a tail entry each, 36 bytes): slices of at most cap trajectories are integrated, their tail
// compacted and replayed, then the node weights are propagated through the network.
static int mlp_grad_run(fpt_ctx *c, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset, double tail_lo,
                        int32_t objective, hipStream_t s, float *d_grad, double *d_G, double *J_out,
                        uint64_t *n_tail_out, unsigned char *sb, size_t cap)
{
    int rc = FPT_OK;
    TailEntry *d_tail = reinterpret_cast<TailEntry *>(sb);
    double *d_N = reinterpret_cast<double *>(sb + 16 * cap);
    double *d_lnw = d_N + cap;
    uint32_t *d_steps = reinterpret_cast<uint32_t *>(d_lnw + cap);
    unsigned long long *cnt = c->d_counters;
    const GridSpec &g = c->grid;
    const size_t n_nodes = (size_t)g.n0 * g.n1;

    HIP_TRY(zero_words(reinterpret_cast<unsigned long long *>(c->d_G), n_nodes, s));
    HIP_TRY(zero_words(reinterpret_cast<unsigned long long *>(c->d_J), 1, s));
    HIP_TRY(zero_words(cnt, 4, s));

    EmParams p{};
    p.inst = c->inst;
    p.inst.acc = c->d_train_acc;
    p.run.dN = dN;
    p.run.sqrt_dN = std::sqrt(dN);
    p.run.key0 = (uint32_t)seed;
    p.run.key1 = (uint32_t)(seed >> 32);
    p.run.chunk = c->opt.chunk ? c->opt.chunk : 128;
    p.cursor = c->cursor;
    p.d_N = d_N;
    p.d_lnw = d_lnw;
    p.d_steps = d_steps;
    const int block = c->opt.block_size ? c->opt.block_size : 1024;
    int grid_em = 0, grid_rp = 0;
    const int n_cells = grid_cells(c->inst);
    rc = occupancy_grid(em_kernel_ptr(c->precision, kBiasMlp, tab_mode(c->inst), c->inst.all_S_pos != 0), block,
                        em_lds_bytes(c->opt.n_bins, c->inst.n_tab, c->precision, n_cells), c->cu_count,
                        c->opt.blocks_per_cu, grid_em);
    if (rc) return rc;
    rc = occupancy_grid(replay_kernel_ptr(c->precision, c->inst.all_S_pos != 0), block,
                        replay_lds_bytes(c->inst.n_tab, c->precision, n_cells, (int)n_nodes), c->cu_count,
                        c->opt.blocks_per_cu, grid_rp);
    if (rc) return rc;
    ReplayParams rp{};
    rp.inst = c->inst;
    rp.run = p.run;
    rp.tail = d_tail;
    rp.n_tail = &cnt[0];
    rp.d_G = c->d_G;
    rp.cursor = &cnt[3];
    rp.mismatch = &cnt[2];
    for (uint64_t done = 0; done < n_traj; done += cap) {
        const uint64_t m = std::min<uint64_t>(cap, n_traj - done);
        HIP_TRY(zero_words(reinterpret_cast<unsigned long long *>(c->d_train_acc), acc_words(c->opt.n_bins), s));
        HIP_TRY(zero_words(c->cursor, 1, s));
        HIP_TRY(zero_words(&cnt[0], 1, s));
        HIP_TRY(zero_words(&cnt[3], 1, s));
        p.traj_offset = traj_offset + done;
        p.n_traj = m;
        HIP_TRY(em_launch(p, c->precision, grid_em, block, s));
        HIP_TRY(mlp_tail_compact(d_N, d_lnw, d_steps, m, traj_offset + done, c->opt.N_ref, tail_lo, d_tail, &cnt[0],
                                 &cnt[1], c->d_J, s));
        HIP_TRY(replay_launch(rp, c->precision, grid_rp, block, s));
    }
    // d_J holds sum_T w^2 = n J: dividing G by it gives d ln J / d theta
    HIP_TRY(mlp_backprop(c->d_params, g, c->d_G, (double)n_traj, objective == FPT_MLP_OBJ_LOG_J ? c->d_J : nullptr,
                         c->d_work, d_grad, s));
    if (d_G) {
        // G / n as documented (scaled copy on the device)
        HIP_TRY(mlp_scale_copy(c->d_G, 1.0 / (double)n_traj, d_G, n_nodes, s));
    }
    if (J_out || n_tail_out) {
        double J = 0.0;
        unsigned long long h_cnt[4] = {0, 0, 0, 0};
        HIP_TRY(hipMemcpyAsync(&J, c->d_J, sizeof J, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(h_cnt, cnt, sizeof h_cnt, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (h_cnt[2] != 0)
            return fail(FPT_EHIP, "%llu replayed trajectories did not end with a passage", (unsigned long long)h_cnt[2]);
        if (J_out) *J_out = J / (double)n_traj;
        if (n_tail_out) *n_tail_out = h_cnt[1];
    }
    return FPT_OK;
}

extern "C" int fpt_mlp_grad(fpt_ctx *c, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                            double tail_lo, int32_t objective, void *hip_stream, float *d_grad, double *d_G,
                            double *J_out, uint64_t *n_tail_out)
{
    int rc = mlp_grad_check(c, n_traj, dN, traj_offset, tail_lo, objective, d_grad);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // per-trajectory scratch: N, ln w (8 B each), steps (4 B) and a tail entry (16 B)
    const size_t slice = std::min<uint64_t>(n_traj, kGradSlice);
    if (slice > c->scratch_cap) {
        if (c->d_scratch) {
            HIP_TRY(hipDeviceSynchronize());
            HIP_TRY(hipFree(c->d_scratch));
            c->d_scratch = nullptr;
            c->scratch_cap = 0;
        }
        const size_t bytes = slice * (8 + 8 + 4 + 16) + 1024;
        if (hipMalloc(&c->d_scratch, bytes) != hipSuccess) {
            c->d_scratch = nullptr;
            return fail(FPT_ENOMEM, "gradient scratch of %zu bytes", bytes);
        }
        c->scratch_cap = slice;
    }
    return mlp_grad_run(c, n_traj, dN, seed, traj_offset, tail_lo, objective, s, d_grad, d_G, J_out, n_tail_out,
                        static_cast<unsigned char *>(c->d_scratch), c->scratch_cap);
}

// ---------------------------------------------------------------------------
// fpt_mlp_grad without allocation: its per-trajectory scratch is a file-scope device array, one
// copy per GPU the library runs on (held until the process ends), reached through the address
// hipGetSymbolAddress gives on each device.  In host code the array's name is no device address.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocMaxTraj = size_t(1) << 18;
static constexpr size_t kNoAllocBytes = kNoAllocMaxTraj * (16 + 8 + 8 + 4) + 1024;
static_assert(kNoAllocMaxTraj == FPT_MLP_GRAD_NOALLOC_MAX, "the header's limit");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of scratch (the current device must be dev).
static int noalloc_scratch(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= kMaxDevices) return fail(FPT_EUNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return FPT_OK;
}

extern "C" int fpt_mlp_grad_noalloc(fpt_ctx *c, uint64_t n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                                    double tail_lo, int32_t objective, void *hip_stream, float *d_grad,
                                    double *d_G, double *J_out, uint64_t *n_tail_out)
{
    int rc = mlp_grad_check(c, n_traj, dN, traj_offset, tail_lo, objective, d_grad);
    if (rc) return rc;
    if (n_traj > kNoAllocMaxTraj)
        return fail(FPT_EINVAL, "n_traj %llu exceeds FPT_MLP_GRAD_NOALLOC_MAX (%zu): the static scratch holds no more",
                    (unsigned long long)n_traj, kNoAllocMaxTraj);
    unsigned char *sb = nullptr;
    rc = noalloc_scratch(c->device, &sb);
    if (rc) return rc;
    return mlp_grad_run(c, n_traj, dN, seed, traj_offset, tail_lo, objective, static_cast<hipStream_t>(hip_stream),
                        d_grad, d_G, J_out, n_tail_out, sb, kNoAllocMaxTraj);
}

extern "C" int fpt_mlp_adam(fpt_ctx *c, const float *d_grad, double lr, double beta1, double beta2, double eps,
                            void *hip_stream)
{
    int rc = mlp_check(c);
    if (rc) return rc;
    if (!d_grad) return fail(FPT_EINVAL, "d_grad is NULL");
    if (!is_finite(lr) || !(lr > 0.0)) return fail(FPT_EINVAL, "lr must be finite and > 0");
    if (!(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0))
        return fail(FPT_EINVAL, "beta1 and beta2 must lie in [0, 1)");
    if (!is_finite(eps) || !(eps > 0.0)) return fail(FPT_EINVAL, "eps must be finite and > 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int t = c->adam_t + 1;
    const double bc1 = 1.0 - std::pow(beta1, (double)t), bc2 = 1.0 - std::pow(beta2, (double)t);
    HIP_TRY(mlp_adam(c->d_params, c->d_adam_m, c->d_adam_v, d_grad, FPT_MLP_NPARAM, lr, beta1, beta2, eps, bc1, bc2,
                     s));
    HIP_TRY(mlp_tabulate(c->d_params, c->grid, c->d_node_a, c->d_grid64, c->d_grid32, s));
    c->adam_t = t;
    return FPT_OK;
}

// ---------------------------------------------------------------------------
// batches of instances: one persistent launch over many contexts
// ---------------------------------------------------------------------------
struct fpt_batch {
    int device = 0, cu_count = 0;
    size_t lds_max = 0;
    int precision = 0, bias_kind = 0;
    bool all_pos = true;
    int n_inst = 0;
    std::vector<fpt_ctx *> ctx;
    int max_bins = 1, max_tab = 1;
    int block = 1024, chunk = 128, item_size = 0;
    bool use_graph = true;
    std::vector<double> est_steps;          // mean steps per trajectory (0 = unknown)
    Inst *d_inst = nullptr, *d_inst_probe = nullptr;
    void *d_probe_acc = nullptr;
    std::vector<size_t> probe_acc_off;
    WorkItem *d_items = nullptr;
    size_t items_cap = 0;
    BatchRun *d_run = nullptr;
    unsigned long long *d_cursors = nullptr;   // [0] tickets, [1 + i] instance i
    WorkItem *h_items = nullptr;            // pinned staging
    size_t h_items_cap = 0;
    BatchRun *h_run = nullptr;              // pinned staging
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;
    int graph_block = 0;
    const void *graph_items = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool ran = false;
};

static void batch_free(fpt_batch *b)
{
    if (!b) return;
    (void)hipDeviceSynchronize();
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_inst) (void)hipFree(b->d_inst);
    if (b->d_inst_probe) (void)hipFree(b->d_inst_probe);
    if (b->d_probe_acc) (void)hipFree(b->d_probe_acc);
    if (b->d_items) (void)hipFree(b->d_items);
    if (b->d_run) (void)hipFree(b->d_run);
    if (b->h_items) (void)hipHostFree(b->h_items);
    if (b->h_run) (void)hipHostFree(b->h_run);
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    if (b->ev_stop) (void)hipEventDestroy(b->ev_stop);
    delete b;
}

extern "C" void fpt_batch_destroy(fpt_batch *b) { batch_free(b); }

extern "C" int fpt_batch_create(fpt_ctx *const *ctx, int32_t n_inst, const fpt_batch_options *opts, fpt_batch **out)
{
    if (!out) return fail(FPT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx || n_inst < 1) return fail(FPT_EINVAL, "need at least one context");
    fpt_batch_options o{};
    if (opts) o = *opts;
    if (o.block_size != 0 && (o.block_size < 64 || o.block_size > 1024 || o.block_size % 64))
        return fail(FPT_EINVAL, "block_size must be a multiple of 64 in 64..1024");
    if (o.chunk != 0 && (o.chunk < 4 || o.chunk % 4)) return fail(FPT_EINVAL, "chunk must be a positive multiple of 4");
    if (o.item_size < 0) return fail(FPT_EINVAL, "item_size must be >= 0");
    for (int i = 0; i < n_inst; ++i) {
        if (!ctx[i]) return fail(FPT_EINVAL, "context %d is NULL", i);
        if (ctx[i]->device != ctx[0]->device) return fail(FPT_EINVAL, "contexts live on different devices");
        if (ctx[i]->precision != ctx[0]->precision) return fail(FPT_EINVAL, "contexts mix FP64 and FP32 state");
        if (ctx[i]->inst.bias_kind == kBiasMlp) return fail(FPT_EINVAL, "a batch cannot hold a learned bias");
        if (ctx[i]->inst.noise_dim == 2) return fail(FPT_EINVAL, "a batch cannot hold 2D noise");
        if (ctx[i]->inst.pot_kind == kPotGaussianBump) return fail(FPT_EINVAL, "a batch cannot hold the Gaussian bump");
        if (ctx[i]->inst.tab_axis) return fail(FPT_EINVAL, "a batch cannot hold a time-indexed table");
    }
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != ctx[0]->device) return fail(FPT_ESTATE, "current device differs from the contexts'");
    fpt_batch *b = new (std::nothrow) fpt_batch();
    if (!b) return fail(FPT_ENOMEM, "host allocation failed");
    b->device = ctx[0]->device;
    b->cu_count = ctx[0]->cu_count;
    b->lds_max = ctx[0]->lds_per_block_max;
    b->precision = ctx[0]->precision;
    b->n_inst = n_inst;
    b->ctx.assign(ctx, ctx + n_inst);
    b->est_steps.assign(n_inst, 0.0);
    b->bias_kind = FPT_BIAS_NONE;
    std::vector<Inst> h(n_inst), hp(n_inst);
    size_t probe_bytes = 0;
    for (int i = 0; i < n_inst; ++i) {
        const Inst &I = ctx[i]->inst;
        h[i] = I;
        if (I.bias_kind == FPT_BIAS_CONST) b->bias_kind = FPT_BIAS_CONST;
        b->all_pos = b->all_pos && I.all_S_pos;
        b->max_bins = std::max(b->max_bins, I.hist.n_bins);
        b->max_tab = std::max(b->max_tab, I.n_tab);
        b->probe_acc_off.push_back(probe_bytes);
        probe_bytes += acc_bytes(I.hist.n_bins);
    }
    if (em_lds_bytes(b->max_bins, b->max_tab, b->precision, 0) > b->lds_max) {
        batch_free(b);
        return fail(FPT_EINVAL, "largest table and histogram do not fit in LDS");
    }
    b->block = o.block_size ? o.block_size : 1024;
    b->chunk = o.chunk ? o.chunk : 128;
    b->item_size = o.item_size;
    b->use_graph = o.use_graph != 0;
    hipError_t e = hipMalloc(&b->d_inst, sizeof(Inst) * n_inst);
    if (e == hipSuccess) e = hipMalloc(&b->d_inst_probe, sizeof(Inst) * n_inst);
    if (e == hipSuccess) e = hipMalloc(&b->d_probe_acc, probe_bytes);
    if (e == hipSuccess) e = hipMalloc(&b->d_run, 128 + sizeof(unsigned long long) * (1 + (size_t)n_inst));
    if (e == hipSuccess) e = hipHostMalloc(&b->h_run, sizeof(BatchRun));
    if (e == hipSuccess) e = hipEventCreate(&b->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&b->ev_stop);
    if (e == hipSuccess) {
        static_assert(sizeof(BatchRun) <= 128, "run parameters and cursors share one allocation");
        b->d_cursors = reinterpret_cast<unsigned long long *>(reinterpret_cast<unsigned char *>(b->d_run) + 128);
        for (int i = 0; i < n_inst; ++i) {
            hp[i] = h[i];
            hp[i].acc = static_cast<unsigned char *>(b->d_probe_acc) + b->probe_acc_off[i];
        }
        e = hipMemcpy(b->d_inst, h.data(), sizeof(Inst) * n_inst, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(b->d_inst_probe, hp.data(), sizeof(Inst) * n_inst, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return hip_fail(e, "fpt_batch_create");
    }
    *out = b;
    return FPT_OK;
}

static int ensure_items(fpt_batch *b, size_t n)
{
    if (n > b->items_cap) {
        if (b->d_items) HIP_TRY(hipFree(b->d_items));
        b->d_items = nullptr;
        size_t cap = std::max<size_t>(n, 2 * b->items_cap);
        HIP_TRY(hipMalloc(&b->d_items, sizeof(WorkItem) * cap));
        b->items_cap = cap;
    }
    if (n > b->h_items_cap) {
        if (b->h_items) HIP_TRY(hipHostFree(b->h_items));
        b->h_items = nullptr;
        size_t cap = std::max<size_t>(n, 2 * b->h_items_cap);
        HIP_TRY(hipHostMalloc(&b->h_items, sizeof(WorkItem) * cap));
        b->h_items_cap = cap;
    }
    return FPT_OK;
}

// Default ticket size: whole trajectories per lane (1..16 per lane of a block), as many as give
// about 32 tickets per resident block in total.
static int default_item_size(const fpt_batch *b, const uint64_t *n_traj, int block)
{
    uint64_t total = 0;
    for (int i = 0; i < b->n_inst; ++i) total += n_traj[i];
    int per_cu = 1;
    const void *fn = batch_kernel_ptr(b->precision, b->bias_kind, b->all_pos);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, block,
                                                     em_lds_bytes(b->max_bins, b->max_tab, b->precision, 0)) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    const double blocks = (double)per_cu * (double)b->cu_count;
    const double per_lane = (double)total / (32.0 * blocks * (double)block);
    const int k = (int)std::max(1.0, std::min(16.0, std::floor(per_lane)));
    return k * block;
}

// The work list of a run: tickets, then one entry per instance (longest estimated cost first);
// every entry of instance i covers its whole range [traj_offset, traj_offset + n_traj[i]).  There
// are as many tickets in total as item_size-sized slices, shared among the instances in proportion
// to their estimated cost (mean steps x trajectories; at least one each) and interleaved by
// stride: ticket k of instance i has the key (k + 1/2)/T_i, so that any prefix of the list holds
// the instances in proportion to their tickets.  n_tickets receives the number of tickets.
static std::vector<WorkItem> make_items(const fpt_batch *b, const uint64_t *n_traj, uint64_t traj_offset,
                                        int item_size, uint64_t &n_tickets)
{
    std::vector<int> live;
    std::vector<double> cost(b->n_inst, 0.0);
    double total_cost = 0.0;
    uint64_t slices = 0;
    for (int i = 0; i < b->n_inst; ++i) {
        if (n_traj[i] == 0) continue;
        live.push_back(i);
        cost[i] = (b->est_steps[i] > 0.0 ? b->est_steps[i] : 1.0) * (double)n_traj[i];
        total_cost += cost[i];
        slices += (n_traj[i] + (uint64_t)item_size - 1) / (uint64_t)item_size;
    }
    struct Key {
        double key, cost;
        int inst;
    };
    std::vector<Key> keys;
    for (int i : live) {
        const uint64_t T = std::max<uint64_t>(1, (uint64_t)std::llround((double)slices * cost[i] / total_cost));
        for (uint64_t k = 0; k < T; ++k) keys.push_back({((double)k + 0.5) / (double)T, cost[i], i});
    }
    std::stable_sort(keys.begin(), keys.end(), [](const Key &x, const Key &y) {
        return x.key < y.key || (x.key == y.key && x.cost > y.cost);
    });
    std::vector<WorkItem> items;
    items.reserve(keys.size() + live.size());
    auto entry = [&](int i) {
        WorkItem w{};
        w.inst = (uint32_t)i;
        w.begin = traj_offset;
        w.count = n_traj[i];
        return w;
    };
    for (const Key &k : keys) items.push_back(entry(k.inst));
    n_tickets = keys.size();
    std::stable_sort(live.begin(), live.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    for (int i : live) items.push_back(entry(i));
    return items;
}

// One persistent launch over `items` with descriptors `d_inst` (direct, or through a captured graph).
static int batch_launch_items(fpt_batch *b, const std::vector<WorkItem> &items, uint64_t n_tickets,
                              const Inst *d_inst, double dN, uint64_t seed, int block, int chunk, hipStream_t s,
                              bool graph)
{
    int rc = ensure_items(b, items.size());
    if (rc) return rc;
    if (b->ran) HIP_TRY(hipEventSynchronize(b->ev_stop));   // the previous launch has read its items
    std::copy(items.begin(), items.end(), b->h_items);
    b->h_run->run.dN = dN;
    b->h_run->run.sqrt_dN = std::sqrt(dN);
    b->h_run->run.key0 = (uint32_t)seed;
    b->h_run->run.key1 = (uint32_t)(seed >> 32);
    b->h_run->run.chunk = chunk;
    b->h_run->n_items = n_tickets;
    b->h_run->n_inst = items.size() - n_tickets;
    HIP_TRY(hipMemcpyAsync(b->d_items, b->h_items, sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(b->d_run, b->h_run, sizeof(BatchRun), hipMemcpyHostToDevice, s));
    const void *fn = batch_kernel_ptr(b->precision, b->bias_kind, b->all_pos);
    int grid = 0;
    rc = occupancy_grid(fn, block, em_lds_bytes(b->max_bins, b->max_tab, b->precision, 0), b->cu_count, 0, grid);
    if (rc) return rc;
    if (graph) {
        if (!b->gexec || b->graph_stream != s || b->graph_block != block || b->graph_items != b->d_items) {
            if (b->gexec) HIP_TRY(hipGraphExecDestroy(b->gexec));
            if (b->graph) HIP_TRY(hipGraphDestroy(b->graph));
            b->gexec = nullptr;
            b->graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            hipError_t e1 = zero_words(b->d_cursors, 1 + (size_t)b->n_inst, s);
            hipError_t e2 = batch_launch(b->precision, b->bias_kind, b->all_pos, d_inst, b->d_items, b->d_run,
                                         b->d_cursors, b->max_bins, b->max_tab, grid, block, s);
            hipError_t e3 = hipStreamEndCapture(s, &b->graph);
            if (e1 != hipSuccess) return hip_fail(e1, "capture: cursor reset");
            if (e2 != hipSuccess) return hip_fail(e2, "capture: batch kernel");
            if (e3 != hipSuccess) return hip_fail(e3, "hipStreamEndCapture");
            HIP_TRY(hipGraphInstantiate(&b->gexec, b->graph, nullptr, nullptr, 0));
            b->graph_stream = s;
            b->graph_block = block;
            b->graph_items = b->d_items;
        }
        HIP_TRY(hipEventRecord(b->ev_start, s));
        HIP_TRY(hipGraphLaunch(b->gexec, s));
        HIP_TRY(hipEventRecord(b->ev_stop, s));
    } else {
        HIP_TRY(zero_words(b->d_cursors, 1 + (size_t)b->n_inst, s));
        HIP_TRY(hipEventRecord(b->ev_start, s));
        HIP_TRY(batch_launch(b->precision, b->bias_kind, b->all_pos, d_inst, b->d_items, b->d_run,
                             b->d_cursors, b->max_bins, b->max_tab, grid, block, s));
        HIP_TRY(hipEventRecord(b->ev_stop, s));
    }
    b->ran = true;
    return FPT_OK;
}

static int check_batch_run(fpt_batch *b, const uint64_t *n_traj, double dN, uint64_t traj_offset)
{
    if (!b || !n_traj) return fail(FPT_EINVAL, "NULL argument");
    if (!(dN > 0.0) || !is_finite(dN)) return fail(FPT_EINVAL, "dN must be finite and > 0");
    for (int i = 0; i < b->n_inst; ++i)
        if (traj_offset + n_traj[i] < traj_offset) return fail(FPT_EINVAL, "trajectory range overflows 64 bits");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != b->device) return fail(FPT_ESTATE, "current device differs from the batch's");
    return FPT_OK;
}

extern "C" int fpt_batch_run(fpt_batch *b, const uint64_t *n_traj, double dN, uint64_t seed, uint64_t traj_offset,
                             void *hip_stream)
{
    int rc = check_batch_run(b, n_traj, dN, traj_offset);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int item_size = b->item_size ? b->item_size : default_item_size(b, n_traj, b->block);
    uint64_t n_tickets = 0;
    std::vector<WorkItem> items = make_items(b, n_traj, traj_offset, item_size, n_tickets);
    if (items.empty()) return FPT_OK;
    // graph capture needs a stream other than the legacy null stream
    rc = batch_launch_items(b, items, n_tickets, b->d_inst, dN, seed, b->block, b->chunk, s,
                            b->use_graph && s != nullptr);
    if (rc) return rc;
    for (int i = 0; i < b->n_inst; ++i) {
        fpt_ctx *c = b->ctx[i];
        c->n_traj_total += n_traj[i];
        c->ran = false;             // no kernel time of its own
        // the batch wrote the accumulators: the context's reads wait for this stream
        HIP_TRY(hipEventRecord(c->ev_done, s));
        c->pending = true;
    }
    return FPT_OK;
}

extern "C" int fpt_batch_last_ms(fpt_batch *b, double *ms)
{
    if (!b || !ms) return fail(FPT_EINVAL, "NULL argument");
    if (!b->ran) return fail(FPT_ESTATE, "no batch run recorded");
    HIP_TRY(hipEventSynchronize(b->ev_stop));
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, b->ev_start, b->ev_stop));
    *ms = (double)f;
    return FPT_OK;
}

extern "C" int fpt_batch_config(fpt_batch *b, int32_t *block_size, int32_t *chunk)
{
    if (!b) return fail(FPT_EINVAL, "NULL argument");
    if (block_size) *block_size = b->block;
    if (chunk) *chunk = b->chunk;
    return FPT_OK;
}

// Steps taken per instance in the probe accumulators (and zero them).
static int probe_steps(fpt_batch *b, std::vector<uint64_t> &steps)
{
    steps.assign(b->n_inst, 0);
    for (int i = 0; i < b->n_inst; ++i) {
        const int nb = b->ctx[i]->inst.hist.n_bins + 2;
        unsigned long long w = 0;
        const unsigned char *acc = static_cast<unsigned char *>(b->d_probe_acc) + b->probe_acc_off[i];
        HIP_TRY(hipMemcpy(&w, acc + sizeof(unsigned long long) * (nb + 2), sizeof w, hipMemcpyDeviceToHost));
        steps[i] = w;
    }
    size_t total = b->probe_acc_off.back() + acc_bytes(b->ctx.back()->inst.hist.n_bins);
    HIP_TRY(hipMemset(b->d_probe_acc, 0, total));
    return FPT_OK;
}

static std::string tune_key(const fpt_batch *b)
{
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
    char buf[256];
    // "t2": the probe layout; entries written by an older probe do not match
    snprintf(buf, sizeof buf, "t2/%s/cu%d/prec%d/bias%d/pos%d/inst%d/tab%d/bins%d", arch.c_str(), b->cu_count,
             b->precision, b->bias_kind, b->all_pos ? 1 : 0, b->n_inst, b->max_tab, b->max_bins);
    for (char &ch : buf)
        if (ch == ' ') ch = '_';
    return buf;
}

extern "C" int fpt_batch_autotune(fpt_batch *b, const uint64_t *n_traj, double dN, uint64_t seed,
                                  const char *cache_path, void *hip_stream)
{
    int rc = check_batch_run(b, n_traj, dN, 0);
    if (rc) return rc;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const std::string key = tune_key(b);
    if (cache_path) {
        FILE *f = fopen(cache_path, "r");
        if (f) {
            char k[256];
            int blk = 0, chk = 0;
            bool found = false;
            while (fscanf(f, "%255s %d %d", k, &blk, &chk) == 3)
                if (key == k && blk >= 64 && blk <= 1024 && blk % 64 == 0 && chk >= 4 && chk % 4 == 0) {
                    b->block = blk;
                    b->chunk = chk;
                    found = true;
                }
            fclose(f);
            if (found) return FPT_OK;
        }
    }
    // probe: one trajectory per lane of a full grid, spread over the instances in proportion to
    // their counts, with a step cap so that each probe launch stays short; the probe's results
    // go to private accumulators and trajectory indices beyond 2^62.
    std::vector<Inst> hp(b->n_inst);
    HIP_TRY(hipMemcpy(hp.data(), b->d_inst_probe, sizeof(Inst) * b->n_inst, hipMemcpyDeviceToHost));
    const uint32_t probe_cap = 1u << 15;
    for (Inst &I : hp) I.max_steps = std::min(I.max_steps, probe_cap);
    HIP_TRY(hipMemcpy(b->d_inst_probe, hp.data(), sizeof(Inst) * b->n_inst, hipMemcpyHostToDevice));
    double total = 0.0;
    for (int i = 0; i < b->n_inst; ++i) total += (double)n_traj[i];
    if (!(total > 0.0)) return fail(FPT_EINVAL, "no trajectories to tune on");
    // enough probe trajectories for about 8 one-trajectory-per-lane items per CU at block 1024
    // (fewer items than resident blocks would leave CUs idle and bias the probe to small blocks)
    const double lanes = (double)b->cu_count * 8192.0;
    std::vector<uint64_t> probe_n(b->n_inst);
    for (int i = 0; i < b->n_inst; ++i)
        probe_n[i] = n_traj[i] ? std::max<uint64_t>(64, (uint64_t)(lanes * (double)n_traj[i] / total)) : 0;
    std::vector<uint64_t> steps;
    rc = probe_steps(b, steps);   // zero
    if (rc) return rc;
    const int blocks[] = {256, 512, 1024};
    const int chunks[] = {32, 64, 128, 256};
    double best = -1.0;
    int best_block = b->block, best_chunk = b->chunk;
    const uint64_t probe_offset = 1ull << 62;
    for (int blk : blocks)
        for (int chk : chunks) {
            uint64_t n_tickets = 0;
            std::vector<WorkItem> items = make_items(b, probe_n.data(), probe_offset, blk, n_tickets);
            rc = batch_launch_items(b, items, n_tickets, b->d_inst_probe, dN, seed, blk, chk, s, false);
            if (rc) return rc;
            double ms = 0.0;
            rc = fpt_batch_last_ms(b, &ms);
            if (rc) return rc;
            rc = probe_steps(b, steps);
            if (rc) return rc;
            double n_steps = 0.0;
            for (uint64_t v : steps) n_steps += (double)v;
            const double rate = n_steps / std::max(ms, 1e-3);
            if (rate > best) {
                best = rate;
                best_block = blk;
                best_chunk = chk;
            }
        }
    b->block = best_block;
    b->chunk = best_chunk;
    // mean steps per trajectory of each instance under its own cap, for the work order
    for (int i = 0; i < b->n_inst; ++i) hp[i].max_steps = b->ctx[i]->inst.max_steps;
    HIP_TRY(hipMemcpy(b->d_inst_probe, hp.data(), sizeof(Inst) * b->n_inst, hipMemcpyHostToDevice));
    std::vector<uint64_t> few(b->n_inst);
    for (int i = 0; i < b->n_inst; ++i) few[i] = n_traj[i] ? 64 : 0;
    uint64_t n_tickets = 0;
    std::vector<WorkItem> items = make_items(b, few.data(), probe_offset, 64, n_tickets);
    rc = batch_launch_items(b, items, n_tickets, b->d_inst_probe, dN, seed, best_block, best_chunk, s, false);
    if (rc) return rc;
    HIP_TRY(hipEventSynchronize(b->ev_stop));
    rc = probe_steps(b, steps);
    if (rc) return rc;
    for (int i = 0; i < b->n_inst; ++i) b->est_steps[i] = few[i] ? (double)steps[i] / (double)few[i] : 0.0;
    if (cache_path) {
        FILE *f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s %d %d\n", key.c_str(), best_block, best_chunk);
            fclose(f);
        }
    }
    return FPT_OK;
}

extern "C" const char *fpt_strerror(int status)
{
    switch (status) {
    case FPT_OK: return "success";
    case FPT_EINVAL: return "invalid argument";
    case FPT_ENOMEM: return "out of memory";
    case FPT_EHIP: return "HIP runtime error";
    case FPT_ESTATE: return "invalid state";
    case FPT_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
    }
}

extern "C" const char *fpt_last_error(void) { return g_last_error.c_str(); }

namespace fpt {
// The last-error message and status of the C ABI, for the other translation units.
int report_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace fpt
