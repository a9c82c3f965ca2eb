// fpt_em.hip -- Euler-Maruyama first-passage kernels for gfx950.
//
// One lane integrates one trajectory of the 1D-noise Langevin system in
// (phi, pi = dphi/dN) (arXiv:2410.13683, Sec. 4.1, eqs. stochastic_eom_1D and
// importance_sampling_1D_noise_step) with a bias parallel to the noise,
// B = a S (1, tan theta_n) (eq. 2D_1D_noise_diussion_based_bias), and
// accumulates ln w = -sum dA (eqs. weight, weight_A restricted to the noise
// direction: dA = a xi sqrt(dN) + a^2 dN / 2 where S > 0).  A trajectory stops
// at its first passage through phi_end; N is interpolated linearly in phi over
// the crossing step.  deltaN = N - N_ref goes into a per-block LDS histogram
// that is flushed to global memory with atomics when the block ends.
//
// Work distribution: a persistent grid; each wave claims trajectories from a
// global cursor with one atomic per refill (ballot + popcount + mbcnt), runs
// `chunk` steps, retires the lanes whose trajectory ended, and refills them.
// New trajectories only start at chunk boundaries and chunks are a multiple of
// 4 steps, so every active lane of a wave is at the same step modulo 4 and the
// Philox call that feeds four steps is taken by the whole wave at once.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed, counter =
// (n >> 2, traj lo, traj hi, instance); u = (w + 1/2) 2^-32; Box-Muller pairs
// (u0, u1) -> steps 4m, 4m+1 and (u2, u3) -> steps 4m+2, 4m+3.
//
// Two state precisions: FP64 (phi, pi, ln w in double) and FP32 state (the
// distance x = phi - phi_end and pi each held as an unevaluated pair of floats
// hi + lo, increments computed in FP32 from the hi parts, uniforms
// fl32(w) 2^-32 + 2^-33 and hardware sin/cos/log; ln w, the crossing
// interpolation and the histogram stay FP64).
#include "internal.hpp"

#include <hip/hip_runtime.h>
#include <math.h>

namespace fpt {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                              uint32_t k0, uint32_t k1, uint32_t w[4])
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c0;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    w[0] = c0; w[1] = c1; w[2] = c2; w[3] = c3;
}

// Box-Muller in FP64 on uniforms (w + 1/2) 2^-32 (exact in double).
__device__ __forceinline__ void box_muller64(uint32_t wa, uint32_t wb, double &za, double &zb)
{
    const double ua = fma((double)wa, 0x1p-32, 0x1p-33);
    const double ub = fma((double)wb, 0x1p-32, 0x1p-33);
    const double rho = sqrt(-2.0 * log(ua));
    double s, c;
    sincospi(2.0 * ub, &s, &c);
    za = rho * c;
    zb = rho * s;
}

// Box-Muller in FP32 on uniforms fl32(w) 2^-32 + 2^-33: the same uniform as the
// FP64 path, rounded to 24 significant bits (relative, not absolute, resolution,
// so the radius stays accurate for small u).  Never 0; at most 1.0f, where the
// radius is 0.  v_log_f32 returns log2, v_sin_f32 / v_cos_f32 take turns.
__device__ __forceinline__ void box_muller32(uint32_t wa, uint32_t wb, float &za, float &zb)
{
    const float ua = fmaf((float)wa, 0x1p-32f, 0x1p-33f);
    const float ub = fmaf((float)wb, 0x1p-32f, 0x1p-33f);
    const float rho = __builtin_sqrtf(fmaxf(-1.3862943611198906f * __builtin_amdgcn_logf(ua), 0.0f));  // -2 ln u
    za = rho * __builtin_amdgcn_cosf(ub);
    zb = rho * __builtin_amdgcn_sinf(ub);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Wave-aggregated claim of trajectories from the global cursor.  Must be
// reached by every lane of the wave.  Returns true in lanes that got one.
__device__ __forceinline__ bool claim(bool need, uint64_t &rel, unsigned long long *cursor, uint64_t n_traj,
                                      bool &exhausted)
{
    const uint64_t mask = __ballot(need && !exhausted);
    if (mask == 0) return false;
    const uint32_t cnt = (uint32_t)__popcll(mask);
    const int leader = __ffsll((unsigned long long)mask) - 1;
    unsigned long long base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(cursor, (unsigned long long)cnt);
    const uint32_t b_lo = (uint32_t)__shfl((int)(uint32_t)base, leader);
    const uint32_t b_hi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), leader);
    const uint64_t b = ((uint64_t)b_hi << 32) | b_lo;
    if (b + cnt >= n_traj) exhausted = true;
    if (need) {
        const uint64_t me = b + lanes_below(mask);
        if (me < n_traj) {
            rel = me;
            return true;
        }
    }
    return false;
}

struct LdsAcc {
    unsigned long long *cnt;  // nb + 4
    double *sum;              // 4 nb + 4
    int nb;
};

__device__ __forceinline__ LdsAcc lds_acc(unsigned char *smem, int n_bins)
{
    LdsAcc a;
    a.nb = n_bins + 2;
    a.cnt = reinterpret_cast<unsigned long long *>(smem);
    a.sum = reinterpret_cast<double *>(a.cnt + a.nb + 4);
    return a;
}

__device__ __forceinline__ int bin_of(const HistSpec &h, double x)
{
    double t;
    if (h.bins_kind == kBinsLinear) t = (x - h.lo) * h.scale;
    else t = (x > 0.0) ? log(x / h.lo) * h.scale : -1.0;
    if (!(t >= 0.0)) return 0;
    if (t >= (double)h.n_bins) return h.n_bins + 1;
    return (int)floor(t) + 1;
}

// Retire one finished trajectory: per-trajectory outputs and LDS histogram.
__device__ __forceinline__ void retire(const EmParams &p, const LdsAcc &a, uint64_t rel, uint32_t status,
                                       uint32_t n_steps, double N, double lnw)
{
    if (p.d_N) p.d_N[rel] = N;
    if (p.d_lnw) p.d_lnw[rel] = lnw;
    if (p.d_steps) p.d_steps[rel] = n_steps | status;
    if (status & kFlagCensored) {
        atomicAdd(&a.cnt[a.nb + 0], 1ull);
    } else if (status & kFlagEndedEarly) {
        atomicAdd(&a.cnt[a.nb + 1], 1ull);
    } else {
        const int b = bin_of(p.hist, N - p.hist.N_ref);
        const double w = exp(lnw);
        atomicAdd(&a.cnt[b], 1ull);
        atomicAdd(&a.sum[b], w);
        atomicAdd(&a.sum[a.nb + b], w * w);
        atomicAdd(&a.sum[2 * a.nb + b], lnw);
        atomicAdd(&a.sum[3 * a.nb + b], lnw * lnw);
        double *tot = a.sum + 4 * a.nb;
        atomicAdd(&tot[0], w);
        atomicAdd(&tot[1], w * w);
        atomicAdd(&tot[2], w * N);
        atomicAdd(&tot[3], w * N * N);
    }
}

__device__ __forceinline__ void zero_lds_acc(const LdsAcc &a)
{
    for (int i = threadIdx.x; i < a.nb + 4; i += blockDim.x) a.cnt[i] = 0ull;
    for (int i = threadIdx.x; i < 4 * a.nb + 4; i += blockDim.x) a.sum[i] = 0.0;
}

__device__ __forceinline__ void flush_lds_acc(const LdsAcc &a, void *global)
{
    unsigned long long *gc = reinterpret_cast<unsigned long long *>(global);
    double *gs = reinterpret_cast<double *>(gc + a.nb + 4);
    for (int i = threadIdx.x; i < a.nb + 4; i += blockDim.x)
        if (a.cnt[i]) atomicAdd(&gc[i], a.cnt[i]);
    for (int i = threadIdx.x; i < 4 * a.nb + 4; i += blockDim.x)
        if (a.sum[i] != 0.0) unsafeAtomicAdd(&gs[i], a.sum[i]);
}

// ---------------------------------------------------------------------------
// FP64 state
// ---------------------------------------------------------------------------
template <int BIAS, bool TAB>
__global__ void __launch_bounds__(1024) em_fp64_kernel(EmParams p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsAcc acc = lds_acc(smem, p.hist.n_bins);
    double *l_S = acc.sum + 4 * acc.nb + 4;
    double *l_t = l_S + p.n_tab;
    zero_lds_acc(acc);
    if (TAB) {
        for (int i = threadIdx.x; i < p.n_tab; i += blockDim.x) {
            l_S[i] = p.tab_S[i];
            l_t[i] = p.tab_t[i];
        }
    }
    __syncthreads();

    const double S0 = p.tab_S[0], t0 = p.tab_t[0];
    const double dN = p.dN, sqrt_dN = p.sqrt_dN;
    const double a = (BIAS == kBiasConst) ? p.A : 0.0;
    const double half_a2_dN = 0.5 * a * a * dN;
    const double tab_jmax = (double)(p.n_tab - 2);

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, p.cursor, p.n_traj, exhausted);
    double phi = p.phi_in, pi_ = p.pi_in, lnw = 0.0;
    uint32_t n = 0;
    uint64_t steps_acc = 0;

    while (__any(has)) {
        bool active = has;
        uint32_t status = 0, n_out = 0;
        double N_out = 0.0, lnw_out = 0.0;
        for (int k = 0; k < p.chunk; k += 4) {
            if (!__any(active)) break;
            if (active) {
                const uint64_t traj = p.traj_offset + rel;
                uint32_t w[4];
                philox4x32_10(n >> 2, (uint32_t)traj, (uint32_t)(traj >> 32), p.instance, p.key0, p.key1, w);
                double z[4];
                box_muller64(w[0], w[1], z[0], z[1]);
                box_muller64(w[2], w[3], z[2], z[3]);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (active) {
                        if (n == p.max_steps) {
                            active = false;
                            status = kFlagCensored;
                            N_out = __builtin_nan("");
                            lnw_out = lnw;
                            n_out = n;
                        } else {
                            // V'/V
                            double r;
                            if (p.pot_kind == kPotExponential) {
                                r = p.A_plus;
                            } else {
                                const double A = (phi >= p.phi_T) ? p.A_plus : p.A_minus;
                                r = A / (p.V0 + A * (phi - p.phi_T));
                            }
                            // noise amplitude and direction at phi
                            double S, t;
                            if (TAB) {
                                const double x = (phi - p.phi_lo) * p.inv_h;
                                const double jf = fmin(fmax(floor(x), 0.0), tab_jmax);
                                const int jj = (int)jf;
                                const double f = fmin(fmax(x - jf, 0.0), 1.0);
                                S = l_S[jj] + f * (l_S[jj + 1] - l_S[jj]);
                                t = l_t[jj] + f * (l_t[jj + 1] - l_t[jj]);
                            } else {
                                S = S0;
                                t = t0;
                            }
                            const double zs = z[j] * sqrt_dN;
                            const double noise = S * zs;
                            const double aS = a * S;
                            const double phi_n = phi + (pi_ + aS) * dN + noise;
                            const double pi_n = pi_ - (3.0 - 0.5 * pi_ * pi_) * (pi_ + r) * dN + t * (aS * dN + noise);
                            if (BIAS != kBiasNone && S > 0.0) lnw -= a * zs + half_a2_dN;
                            if (phi_n <= p.phi_end) {
                                active = false;
                                status = 0;
                                N_out = (double)n * dN + dN * ((phi - p.phi_end) / (phi - phi_n));
                                lnw_out = lnw;
                                n_out = n + 1;
                            } else if (0.5 * pi_n * pi_n >= 1.0) {
                                active = false;
                                status = kFlagEndedEarly;
                                N_out = (double)(n + 1) * dN;
                                lnw_out = lnw;
                                n_out = n + 1;
                            }
                            phi = phi_n;
                            pi_ = pi_n;
                            n += 1;
                        }
                    }
                }
            }
        }
        if (has && !active) {
            retire(p, acc, rel, status, n_out, N_out, lnw_out);
            steps_acc += n_out;
            has = false;
        }
        if (claim(!has, rel, p.cursor, p.n_traj, exhausted)) {
            has = true;
            phi = p.phi_in;
            pi_ = p.pi_in;
            lnw = 0.0;
            n = 0;
        }
    }
    if (steps_acc) atomicAdd(&acc.cnt[acc.nb + 2], (unsigned long long)steps_acc);
    __syncthreads();
    flush_lds_acc(acc, p.acc);
}

// ---------------------------------------------------------------------------
// FP32 state: x = phi - phi_end and pi as float pairs (hi + lo).
// ---------------------------------------------------------------------------
struct F32Consts {
    float xT_hi, xT_lo;        // phi_T - phi_end as a float pair
    float q_plus, q_minus;     // V0/A_+ and V0/A_-  (1/r = (phi - phi_T) + V0/A)
    float r_exp;               // A_+ for the exponential potential
    float c_tab;               // phi_end - phi_lo
    float inv_h;
    float dN, sqrt_dN;
    float a, a_dN;
};

__device__ __forceinline__ void two_sum_fast(float &hi, float &lo, float d)
{
    // hi + lo += d with |hi| >= |d| (Fast2Sum of hi and d, error folded into lo)
    const float s = hi + d;
    const float e = d - (s - hi);
    hi = s;
    lo += e;
}

template <int BIAS, bool TAB>
__global__ void __launch_bounds__(1024) em_fp32s_kernel(EmParams p, F32Consts c)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsAcc acc = lds_acc(smem, p.hist.n_bins);
    float *l_S = reinterpret_cast<float *>(acc.sum + 4 * acc.nb + 4);
    float *l_t = l_S + p.n_tab;
    zero_lds_acc(acc);
    if (TAB) {
        for (int i = threadIdx.x; i < p.n_tab; i += blockDim.x) {
            l_S[i] = p.tab_Sf[i];
            l_t[i] = p.tab_tf[i];
        }
    }
    __syncthreads();

    const float S0 = p.tab_Sf[0], t0 = p.tab_tf[0];
    const float tab_jmax = (float)(p.n_tab - 2);
    const double x_in = p.phi_in - p.phi_end;
    const float x_in_hi = (float)x_in, x_in_lo = (float)(x_in - (double)x_in_hi);
    const double pi_in = p.pi_in;
    const float pi_in_hi = (float)pi_in, pi_in_lo = (float)(pi_in - (double)pi_in_hi);
    const double dN = p.dN;

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, p.cursor, p.n_traj, exhausted);
    float xh = x_in_hi, xl = x_in_lo, ph = pi_in_hi, pl = pi_in_lo;
    double zsum = 0.0;        // sum of xi over steps with S > 0 (constant bias)
    uint32_t n_on = 0;        // number of such steps
    uint32_t n = 0;
    uint64_t steps_acc = 0;

    while (__any(has)) {
        bool active = has;
        uint32_t status = 0, n_out = 0;
        double N_out = 0.0, zsum_out = 0.0;
        uint32_t non_out = 0;
        for (int k = 0; k < p.chunk; k += 4) {
            if (!__any(active)) break;
            if (active) {
                const uint64_t traj = p.traj_offset + rel;
                uint32_t w[4];
                philox4x32_10(n >> 2, (uint32_t)traj, (uint32_t)(traj >> 32), p.instance, p.key0, p.key1, w);
                float z[4];
                box_muller32(w[0], w[1], z[0], z[1]);
                box_muller32(w[2], w[3], z[2], z[3]);
                float zpart = 0.0f;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (active) {
                        if (n == p.max_steps) {
                            active = false;
                            status = kFlagCensored;
                            N_out = __builtin_nan("");
                            zsum_out = zsum + (double)zpart;
                            non_out = n_on;
                            n_out = n;
                        } else {
                            // phi - phi_T as an accurate float: (xh - xT_hi) + (xl - xT_lo)
                            const float dT = (xh - c.xT_hi) + (xl - c.xT_lo);
                            float r;
                            if (p.pot_kind == kPotExponential) r = c.r_exp;
                            else r = __builtin_amdgcn_rcpf(dT + ((dT >= 0.0f) ? c.q_plus : c.q_minus));
                            float S, t;
                            if (TAB) {
                                const float u = (xh + c.c_tab) * c.inv_h;
                                const float jf = fminf(fmaxf(floorf(u), 0.0f), tab_jmax);
                                const int jj = (int)jf;
                                const float f = fminf(fmaxf(u - jf, 0.0f), 1.0f);
                                S = l_S[jj] + f * (l_S[jj + 1] - l_S[jj]);
                                t = l_t[jj] + f * (l_t[jj + 1] - l_t[jj]);
                            } else {
                                S = S0;
                                t = t0;
                            }
                            const float noise = S * (z[j] * c.sqrt_dN);
                            const float aS = c.a * S;
                            const float dx = (ph + aS) * c.dN + noise;
                            const float dpi = -(3.0f - 0.5f * ph * ph) * (ph + r) * c.dN + t * (aS * c.dN + noise);
                            if (BIAS != kBiasNone && S > 0.0f) {
                                zpart += z[j];
                                n_on += 1;
                            }
                            const float xh_old = xh, xl_old = xl;
                            two_sum_fast(xh, xl, dx);
                            two_sum_fast(ph, pl, dpi);
                            if (xh + xl <= 0.0f) {
                                active = false;
                                status = 0;
                                const double x0 = (double)xh_old + (double)xl_old;
                                const double x1 = (double)xh + (double)xl;
                                N_out = (double)n * dN + dN * (x0 / (x0 - x1));
                                zsum_out = zsum + (double)zpart;
                                non_out = n_on;
                                n_out = n + 1;
                            } else if (0.5f * ph * ph >= 1.0f) {
                                active = false;
                                status = kFlagEndedEarly;
                                N_out = (double)(n + 1) * dN;
                                zsum_out = zsum + (double)zpart;
                                non_out = n_on;
                                n_out = n + 1;
                            }
                            n += 1;
                        }
                    }
                }
                zsum += (double)zpart;
                // renormalise the pairs once per group of four steps
                {
                    const float s = xh + xl;
                    xl = xl - (s - xh);
                    xh = s;
                    const float q = ph + pl;
                    pl = pl - (q - ph);
                    ph = q;
                }
            }
        }
        if (has && !active) {
            const double lnw = (BIAS == kBiasNone)
                                   ? 0.0
                                   : -p.A * p.sqrt_dN * zsum_out - (double)non_out * (0.5 * p.A * p.A * dN);
            retire(p, acc, rel, status, n_out, N_out, lnw);
            steps_acc += n_out;
            has = false;
        }
        if (claim(!has, rel, p.cursor, p.n_traj, exhausted)) {
            has = true;
            xh = x_in_hi;
            xl = x_in_lo;
            ph = pi_in_hi;
            pl = pi_in_lo;
            zsum = 0.0;
            n_on = 0;
            n = 0;
        }
    }
    if (steps_acc) atomicAdd(&acc.cnt[acc.nb + 2], (unsigned long long)steps_acc);
    __syncthreads();
    flush_lds_acc(acc, p.acc);
}

__global__ void zero_words_kernel(unsigned long long *ptr, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        ptr[i] = 0ull;
}

F32Consts make_f32_consts(const EmParams &p)
{
    F32Consts c;
    const double xT = p.phi_T - p.phi_end;
    c.xT_hi = (float)xT;
    c.xT_lo = (float)(xT - (double)c.xT_hi);
    c.q_plus = (float)(p.V0 / p.A_plus);
    c.q_minus = (float)(p.V0 / p.A_minus);
    c.r_exp = (float)p.A_plus;
    c.c_tab = (float)(p.phi_end - p.phi_lo);
    c.inv_h = (float)p.inv_h;
    c.dN = (float)p.dN;
    c.sqrt_dN = (float)p.sqrt_dN;
    c.a = (p.bias_kind == kBiasConst) ? (float)p.A : 0.0f;
    c.a_dN = c.a * c.dN;
    return c;
}

template <int BIAS, bool TAB>
const void *pick64() { return reinterpret_cast<const void *>(&em_fp64_kernel<BIAS, TAB>); }
template <int BIAS, bool TAB>
const void *pick32() { return reinterpret_cast<const void *>(&em_fp32s_kernel<BIAS, TAB>); }

}  // namespace

size_t em_lds_bytes(const EmParams &p, int precision)
{
    const size_t acc = acc_bytes(p.hist.n_bins);
    const size_t tab = (p.n_tab > 1) ? (size_t)p.n_tab * 2 * (precision == 0 ? 8 : 4) : 0;
    return acc + tab;
}

const void *em_kernel_ptr(const EmParams &p, int precision)
{
    const bool tab = p.n_tab > 1;
    const int b = p.bias_kind;
    if (precision == 0) {
        if (b == kBiasNone) return tab ? pick64<kBiasNone, true>() : pick64<kBiasNone, false>();
        return tab ? pick64<kBiasConst, true>() : pick64<kBiasConst, false>();
    }
    if (b == kBiasNone) return tab ? pick32<kBiasNone, true>() : pick32<kBiasNone, false>();
    return tab ? pick32<kBiasConst, true>() : pick32<kBiasConst, false>();
}

hipError_t em_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream)
{
    const size_t lds = em_lds_bytes(p, precision);
    const bool tab = p.n_tab > 1;
    const int b = p.bias_kind;
    if (precision == 0) {
        if (b == kBiasNone) {
            if (tab) hipLaunchKernelGGL((em_fp64_kernel<kBiasNone, true>), dim3(grid), dim3(block), lds, stream, p);
            else hipLaunchKernelGGL((em_fp64_kernel<kBiasNone, false>), dim3(grid), dim3(block), lds, stream, p);
        } else {
            if (tab) hipLaunchKernelGGL((em_fp64_kernel<kBiasConst, true>), dim3(grid), dim3(block), lds, stream, p);
            else hipLaunchKernelGGL((em_fp64_kernel<kBiasConst, false>), dim3(grid), dim3(block), lds, stream, p);
        }
    } else {
        const F32Consts c = make_f32_consts(p);
        if (b == kBiasNone) {
            if (tab) hipLaunchKernelGGL((em_fp32s_kernel<kBiasNone, true>), dim3(grid), dim3(block), lds, stream, p, c);
            else hipLaunchKernelGGL((em_fp32s_kernel<kBiasNone, false>), dim3(grid), dim3(block), lds, stream, p, c);
        } else {
            if (tab) hipLaunchKernelGGL((em_fp32s_kernel<kBiasConst, true>), dim3(grid), dim3(block), lds, stream, p, c);
            else hipLaunchKernelGGL((em_fp32s_kernel<kBiasConst, false>), dim3(grid), dim3(block), lds, stream, p, c);
        }
    }
    return hipGetLastError();
}

hipError_t zero_words(unsigned long long *ptr, size_t n, hipStream_t stream)
{
    const int block = 256;
    int grid = (int)((n + block - 1) / block);
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid), dim3(block), 0, stream, ptr, n);
    return hipGetLastError();
}

}  // namespace fpt
