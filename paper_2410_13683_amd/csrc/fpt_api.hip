// fpt_api.hip -- the C ABI declared in include/fpt.h: argument validation,
// device memory of a context, launch configuration, histogram read-back, and
// the device kernel that evaluates the Bessel-ansatz noise table.
#include "fpt.h"
#include "internal.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

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

double pot_V(const fpt_potential &p, double phi)
{
    if (p.kind == FPT_POT_EXPONENTIAL) return p.V0 * std::exp(p.A_plus * (phi - p.phi_T));
    return p.V0 + ((phi >= p.phi_T) ? p.A_plus : p.A_minus) * (phi - p.phi_T);
}

int check_potential(const fpt_potential *pot)
{
    if (!pot) return fail(FPT_EINVAL, "potential is NULL");
    if (pot->kind != FPT_POT_PIECEWISE_LINEAR && pot->kind != FPT_POT_EXPONENTIAL)
        return fail(FPT_EINVAL, "unknown potential kind %d", pot->kind);
    const double v[] = {pot->V0, pot->phi_T, pot->A_plus, pot->A_minus, pot->phi_in, pot->pi_in, pot->phi_end};
    for (double x : v)
        if (!is_finite(x)) return fail(FPT_EINVAL, "potential parameters must be finite");
    if (!(pot->V0 > 0.0)) return fail(FPT_EINVAL, "V0 must be > 0");
    if (pot->kind == FPT_POT_PIECEWISE_LINEAR && (pot->A_plus == 0.0 || pot->A_minus == 0.0))
        return fail(FPT_EINVAL, "A_plus and A_minus must be non-zero");
    return FPT_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// noise table kernel: eq. (covariance_constant_nu) with eq. (nu_squared_approximation)
// ---------------------------------------------------------------------------
__global__ void table_bessel_kernel(int kind, double V0, double phi_T, double Ap, double Am, double sigma, int n,
                                    double phi_lo, double h, double *S, double *t, int *bad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const double phi = phi_lo + (double)j * h;
    double V, r1, r2;
    if (kind == FPT_POT_EXPONENTIAL) {
        V = V0 * exp(Ap * (phi - phi_T));
        r1 = Ap;          // V'/V
        r2 = Ap * Ap;     // V''/V
    } else {
        const double A = (phi >= phi_T) ? Ap : Am;
        V = V0 + A * (phi - phi_T);
        r1 = A / V;
        r2 = 0.0;
    }
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
        hipLaunchKernelGGL(table_bessel_kernel, dim3((n + 255) / 256), dim3(256), 0, 0, pot->kind, pot->V0,
                           pot->phi_T, pot->A_plus, pot->A_minus, sigma, n, phi_lo, h, d, d + n, d_bad);
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
// context
// ---------------------------------------------------------------------------
struct fpt_ctx {
    int device = 0;
    int cu_count = 0;
    size_t lds_per_block_max = 0;
    int precision = FPT_FP64;
    fpt_potential pot{};
    fpt_options opt{};
    EmParams base{};
    void *d_mem = nullptr;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_done = nullptr;
    bool ran = false;
    uint64_t n_traj_total = 0;
};

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
    // noise table
    const int nt = table->n;
    if (nt < 1 || nt > FPT_MAX_TABLE) return fail(FPT_EINVAL, "table size %d out of 1..%d", nt, FPT_MAX_TABLE);
    if (!table->S || !table->tan_theta) return fail(FPT_EINVAL, "table arrays are NULL");
    for (int i = 0; i < nt; ++i) {
        if (!is_finite(table->S[i]) || !is_finite(table->tan_theta[i]))
            return fail(FPT_EINVAL, "table entries must be finite");
        if (table->S[i] < 0.0) return fail(FPT_EINVAL, "table S must be >= 0");
    }
    if (nt > 1 && (!is_finite(table->phi_lo) || !is_finite(table->phi_hi) || !(table->phi_hi > table->phi_lo)))
        return fail(FPT_EINVAL, "table needs phi_hi > phi_lo");
    // bias
    fpt_bias b{};
    if (bias) b = *bias;
    if (b.kind != FPT_BIAS_NONE && b.kind != FPT_BIAS_CONST && b.kind != FPT_BIAS_MLP)
        return fail(FPT_EINVAL, "unknown bias kind %d", b.kind);
    if (!is_finite(b.A)) return fail(FPT_EINVAL, "bias amplitude must be finite");
    if (b.kind == FPT_BIAS_MLP) return fail(FPT_EUNSUPPORTED, "learned bias is not available in fpt_create yet");
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
    c->pot = *pot;
    c->opt = o;
    c->precision = o.precision;
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device);
    int lds_max = 0;
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device);
    c->lds_per_block_max = (size_t)lds_max;
    // device memory: FP64 table (nt x double2), FP32 table (nt x float4), cursor, accumulators
    const size_t off_tab32 = sizeof(double) * 2 * nt;
    const size_t off_cursor = (off_tab32 + sizeof(float) * 4 * nt + 255) & ~size_t(255);
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
    for (int i = 0; i < nt; ++i) {
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
    unsigned char *base = static_cast<unsigned char *>(c->d_mem);
    e = hipMemcpy(base, h64.data(), sizeof(double) * 2 * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(base + off_tab32, h32.data(), sizeof(float) * 4 * nt, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(base + off_cursor, 0, 256 + acc_bytes(o.n_bins));
    if (e == hipSuccess) e = hipEventCreate(&c->ev_start);
    if (e == hipSuccess) e = hipEventCreate(&c->ev_stop);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        fpt_destroy(c);
        return hip_fail(e, "fpt_create initialisation");
    }
    EmParams &p = c->base;
    p.pot_kind = pot->kind;
    p.V0 = pot->V0; p.phi_T = pot->phi_T; p.A_plus = pot->A_plus; p.A_minus = pot->A_minus;
    p.phi_in = pot->phi_in; p.pi_in = pot->pi_in; p.phi_end = pot->phi_end;
    p.n_tab = nt;
    p.phi_lo = (nt > 1) ? table->phi_lo : 0.0;
    p.inv_h = (nt > 1) ? (double)(nt - 1) / (table->phi_hi - table->phi_lo) : 0.0;
    p.tab64 = reinterpret_cast<const double2 *>(base);
    p.tab32 = reinterpret_cast<const float4 *>(base + off_tab32);
    p.all_S_pos = all_pos ? 1 : 0;
    p.bias_kind = b.kind;
    p.A = (b.kind == FPT_BIAS_CONST) ? b.A : 0.0;
    p.mlp = nullptr;
    p.mlp_every = 1;
    p.max_steps = (uint32_t)o.max_steps;
    p.hist.bins_kind = o.bins_kind;
    p.hist.n_bins = o.n_bins;
    p.hist.lo = o.lo;
    p.hist.N_ref = o.N_ref;
    p.hist.scale = (o.bins_kind == FPT_BINS_LINEAR) ? (double)o.n_bins / (o.hi - o.lo)
                                                    : (double)o.n_bins / std::log(o.hi / o.lo);
    p.cursor = reinterpret_cast<unsigned long long *>(base + off_cursor);
    p.acc = base + off_acc;
    p.instance = o.instance;
    if (em_lds_bytes(p, c->precision) > c->lds_per_block_max) {
        fpt_destroy(c);
        return fail(FPT_EINVAL, "noise table and histogram do not fit in LDS (%zu > %zu bytes)",
                    em_lds_bytes(p, o.precision), (size_t)lds_max);
    }
    *out = c;
    return FPT_OK;
}

static int launch_config(fpt_ctx *c, const EmParams &p, int &grid, int &block)
{
    block = c->opt.block_size ? c->opt.block_size : 1024;
    int per_cu = c->opt.blocks_per_cu;
    if (per_cu == 0) {
        int occ = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, em_kernel_ptr(p, c->precision), block,
                                                                    em_lds_bytes(p, c->precision));
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        per_cu = occ > 0 ? occ : 1;
    }
    grid = per_cu * c->cu_count;
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
    EmParams p = c->base;
    p.dN = dN;
    p.sqrt_dN = std::sqrt(dN);
    p.key0 = (uint32_t)seed;
    p.key1 = (uint32_t)(seed >> 32);
    p.traj_offset = traj_offset;
    p.n_traj = n_traj;
    p.chunk = c->opt.chunk ? c->opt.chunk : 128;
    p.d_N = d_N;
    p.d_lnw = d_lnw;
    p.d_steps = d_steps;
    int grid = 0, block = 0;
    int rc = launch_config(c, p, grid, block);
    if (rc) return rc;
    HIP_TRY(zero_words(p.cursor, 1, s));
    HIP_TRY(hipEventRecord(c->ev_start, s));
    HIP_TRY(em_launch(p, c->precision, grid, block, s));
    HIP_TRY(hipEventRecord(c->ev_stop, s));
    HIP_TRY(hipEventRecord(c->ev_done, s));
    c->ran = true;
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

extern "C" int fpt_histogram(fpt_ctx *c, fpt_hist *out)
{
    if (!c || !out) return fail(FPT_EINVAL, "NULL argument");
    if (!out->count || !out->sum_w_bin || !out->sum_w2_bin || !out->sum_lnw_bin || !out->sum_lnw2_bin)
        return fail(FPT_EINVAL, "histogram arrays are NULL");
    if (c->ran) HIP_TRY(hipEventSynchronize(c->ev_done));
    const int nb = c->opt.n_bins + 2;
    std::vector<unsigned char> h(acc_bytes(c->opt.n_bins));
    HIP_TRY(hipMemcpy(h.data(), c->base.acc, h.size(), hipMemcpyDeviceToHost));
    const unsigned long long *cnt = reinterpret_cast<const unsigned long long *>(h.data());
    const double *sum = reinterpret_cast<const double *>(cnt + nb + 4);
    for (int i = 0; i < nb; ++i) {
        out->count[i] = cnt[i];
        out->sum_w_bin[i] = sum[i];
        out->sum_w2_bin[i] = sum[nb + i];
        out->sum_lnw_bin[i] = sum[2 * nb + i];
        out->sum_lnw2_bin[i] = sum[3 * nb + i];
    }
    out->n_traj = c->n_traj_total;
    out->n_censored = cnt[nb + 0];
    out->n_ended_early = cnt[nb + 1];
    out->n_steps_total = cnt[nb + 2];
    out->sum_w = sum[4 * nb + 0];
    out->sum_w2 = sum[4 * nb + 1];
    out->sum_wN = sum[4 * nb + 2];
    out->sum_wN2 = sum[4 * nb + 3];
    return FPT_OK;
}

extern "C" int fpt_reset(fpt_ctx *c)
{
    if (!c) return fail(FPT_EINVAL, "context is NULL");
    if (c->ran) HIP_TRY(hipEventSynchronize(c->ev_done));
    HIP_TRY(hipMemset(c->base.acc, 0, acc_bytes(c->opt.n_bins)));
    HIP_TRY(hipDeviceSynchronize());
    c->n_traj_total = 0;
    return FPT_OK;
}

extern "C" void fpt_destroy(fpt_ctx *c)
{
    if (!c) return;
    // teardown errors cannot be reported through a void function
    if (c->ran && c->ev_done) (void)hipEventSynchronize(c->ev_done);
    if (c->ev_start) (void)hipEventDestroy(c->ev_start);
    if (c->ev_stop) (void)hipEventDestroy(c->ev_stop);
    if (c->ev_done) (void)hipEventDestroy(c->ev_done);
    if (c->d_mem) (void)hipFree(c->d_mem);
    delete c;
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
