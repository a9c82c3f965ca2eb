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
// New trajectories only start at chunk boundaries and a chunk is a whole number
// of step groups (FP64: 4 steps, 2 with 2D noise; FP32: 16, except the kernel
// that evaluates the network in the step, 4; a chunk is rounded up to a whole
// group), so every active lane of a wave is at the same step modulo the group
// length and each Philox call (four steps of 1D noise, two of 2D noise) is
// taken by the whole wave at once.
//
// Random numbers: Philox4x32-10 (Salmon et al., SC'11), key = seed, counter =
// (traj lo, n >> 2, traj hi, instance); u = (w + 1/2) 2^-32; Box-Muller pairs
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

#include <type_traits>

// Optional register budget for the Euler-Maruyama kernels (waves per SIMD the
// compiler must leave room for); unset = the compiler's choice.
#ifdef FPT_EM_WAVES_PER_EU
#define FPT_EM_OCCUPANCY __attribute__((amdgpu_waves_per_eu(FPT_EM_WAVES_PER_EU)))
#else
#define FPT_EM_OCCUPANCY
#endif

namespace fpt {
namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;

// a ^ b ^ c in one instruction: gfx950's three-input bitwise op with the XOR
// truth table 0x96 (c is wave-uniform, the round key).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t d;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

// Philox4x32-10 (Salmon et al., SC'11): ten rounds on the counter (c0, c1, c2, c3) with the key
// (k0, k1); a round forms the 64-bit products M0 c0 and M1 c2 and maps the counter to
// (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)), then adds the Weyl
// increments (W0, W1) to the key.  Here the counter is (traj lo, m, traj hi, instance) for a fixed
// trajectory, key and instance word, and only the call index m varies.  It sits in a word that
// round 1 XORs but does not multiply, so every product that does not depend on m is a
// per-trajectory constant: both products of round 1, M1 times round 1's word 2 in round 2, and
// M0 times round 2's word 0 in round 3.  They are computed once when a lane takes a trajectory
// (philox_pre), which leaves rounds 1 to 3 two multiplies in all instead of six.
struct PhiloxPre {
    uint32_t a;     // round 1 output word 0 without m: hi(M1 thi) ^ k0 (the word is a ^ m)
    uint32_t y;     // lo(M0 tlo) ^ round 2's key word 1 (round 2 output word 2 is hi(M0 (a ^ m)) ^ y)
    uint32_t x1k;   // lo(M1 (hi(M0 tlo) ^ inst ^ k1)) ^ round 3's key word 0
    uint32_t z;     // hi(M0 x0) ^ round 3's key word 1, x0 round 2's output word 0 (constant)
    uint32_t w;     // lo(M0 x0): round 3 output word 3
};

__device__ __forceinline__ PhiloxPre philox_pre(uint64_t traj, uint32_t inst, uint32_t k0, uint32_t k1)
{
    const uint64_t p = (uint64_t)kPhiloxM0 * (uint32_t)traj;            // round 1: M0 c0
    const uint64_t q = (uint64_t)kPhiloxM1 * (uint32_t)(traj >> 32);    // round 1: M1 c2
    PhiloxPre r;
    r.a = (uint32_t)(q >> 32) ^ k0;
    const uint32_t d = (uint32_t)(p >> 32) ^ inst ^ k1;                 // round 1 output word 2
    r.y = (uint32_t)p ^ (k1 + kPhiloxW1);
    const uint64_t q2 = (uint64_t)kPhiloxM1 * d;                        // round 2: M1 c2
    const uint32_t x0 = (uint32_t)(q2 >> 32) ^ (uint32_t)q ^ (k0 + kPhiloxW0);
    r.x1k = (uint32_t)q2 ^ (k0 + 2u * kPhiloxW0);
    const uint64_t p3 = (uint64_t)kPhiloxM0 * x0;                       // round 3: M0 c0
    r.z = (uint32_t)(p3 >> 32) ^ (k1 + 2u * kPhiloxW1);
    r.w = (uint32_t)p3;
    return r;
}

// The four output words for call m from the trajectory's PhiloxPre.
__device__ __forceinline__ void philox_call(uint32_t m, const PhiloxPre &q, uint32_t k0, uint32_t k1, uint32_t w[4])
{
    // round 2: M0 (a ^ m); words 0 and 1 are per-trajectory constants
    const uint64_t p2 = (uint64_t)kPhiloxM0 * (q.a ^ m);
    const uint32_t v2 = (uint32_t)(p2 >> 32) ^ q.y;
    const uint32_t v3 = (uint32_t)p2;
    // round 3: M1 v2; M0 times the constant word 0 is precomputed
    const uint64_t q3 = (uint64_t)kPhiloxM1 * v2;
    uint32_t d0 = (uint32_t)(q3 >> 32) ^ q.x1k;
    uint32_t d1 = (uint32_t)q3;
    uint32_t d2 = q.z ^ v3;
    uint32_t d3 = q.w;
    k0 += 3u * kPhiloxW0;
    k1 += 3u * kPhiloxW1;
    // rounds 4 .. 10
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        const uint64_t a = (uint64_t)kPhiloxM0 * d0;
        const uint64_t b = (uint64_t)kPhiloxM1 * d2;
        const uint32_t n0 = xor3((uint32_t)(b >> 32), d1, k0);
        const uint32_t n2 = xor3((uint32_t)(a >> 32), d3, k1);
        d1 = (uint32_t)b;
        d3 = (uint32_t)a;
        d0 = n0;
        d2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    w[0] = d0; w[1] = d1; w[2] = d2; w[3] = d3;
}

// Box-Muller in FP64 on uniforms u = (w + 1/2) 2^-32 (exact in double), table-driven: two
// 256-entry tables in LDS (kBmBytes, staged once per block by stage_bm) replace the library
// log and sincos, each by a table read and a short series.
//   ln u:  u = m 2^e, m in [0.5, 1).  Bucket i (top 8 fraction bits of m) has centre c_i
//          (c_255 = 1, so that u near 1 loses nothing to cancellation), r_i = fl(1/c_i) and
//          L_i = -ln r_i.  Then ln m = L_i + ln(1 + t), t = m r_i - 1, |t| <= 2^-9, and the
//          series to t^5 leaves t^6/6 < 1e-17.
//   2 pi u: (2 w + 1) 2^-33 = (j + 1/2)/256 + d 2^-33, j = w >> 24, d = 2 (w mod 2^24) + 1 - 2^24
//          (an exact integer, |d| < 2^24).  sin and cos of A_j = 2 pi (j + 1/2)/256 come from
//          the table; theta = 2 pi d 2^-33 (|theta| <= pi/256) from series to theta^5 and
//          theta^6 (errors < 1e-17 and < 2e-23), and the angle-addition formulas combine them.
// Both stay far below what per-trajectory agreement to 1e-9 with an FP64 reference needs
// (normals to ~1e-9): the series stop where the next term is below 1e-17.
// Returns xi sqrt(dN) for the two steps of the pair.
constexpr int kBmN = 256;
constexpr size_t kBmBytes = 2 * kBmN * sizeof(double2);

// l_bm[j] = (sin A_j, cos A_j); l_bm[kBmN + i] = (r_i, L_i)
__device__ __forceinline__ void stage_bm(double2 *l_bm)
{
    for (int i = threadIdx.x; i < 2 * kBmN; i += blockDim.x) {
        if (i < kBmN) {
            double sn, cs;
            sincospi((i + 0.5) * (1.0 / 128.0), &sn, &cs);
            l_bm[i] = make_double2(sn, cs);
        } else {
            const int k = i - kBmN;
            const double c = (k == kBmN - 1) ? 1.0 : 0.5 * (1.0 + (k + 0.5) * (1.0 / 256.0));
            const double r = 1.0 / c;
            l_bm[i] = make_double2(r, -log(r));
        }
    }
}

// sqrt(x) for x in [2e-10, 50] (here -2 ln u: never 0, denormal or infinite, so the library's
// scaling and special-case tests are not needed): the hardware reciprocal square root, one
// Goldschmidt step and one residual correction, s = g + (x - g^2) h (within about an ulp).
__device__ __forceinline__ double sqrt_mid(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    return fma(fma(-g, g, x), h, g);
}

__device__ __forceinline__ void box_muller64(uint32_t wa, uint32_t wb, double sqrt_dN, const double2 *l_bm,
                                             double &za, double &zb)
{
    const double ua = fma((double)wa, 0x1p-32, 0x1p-33);
    const double m = __builtin_amdgcn_frexp_mant(ua);        // [0.5, 1)
    const int e = __builtin_amdgcn_frexp_exp(ua);
    const int i = (__double2hiint(m) >> 12) & 0xff;
    const double2 lt = l_bm[kBmN + i];
    const double t = fma(m, lt.x, -1.0);
    double q = fma(t, 0.2, -0.25);
    q = fma(t, q, 1.0 / 3.0);
    q = fma(t, q, -0.5);
    q = fma(t, q, 1.0);
    const double ln_u = fma((double)e, 0x1.62e42fefa39efp-1, fma(t, q, lt.y));   // e ln 2 + L_i + ln(1 + t)
    const double rho = sqrt_mid(-2.0 * ln_u) * sqrt_dN;
    const int d = (int)((wb & 0xffffffu) << 1) + 1 - (1 << 24);
    const double th = (double)d * 0x1.921fb54442d18p-31;                          // 2 pi d 2^-33
    const double th2 = th * th;
    const double sn = th * fma(th2, fma(th2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
    const double cs = fma(th2, fma(th2, fma(th2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
    const double2 sc = l_bm[wb >> 24];
    za = rho * fma(sc.y, cs, -sc.x * sn);      // cos(A + theta)
    zb = rho * fma(sc.x, cs, sc.y * sn);       // sin(A + theta)
}

// Copy a wave-uniform value into a VGPR once, so that a per-lane select between
// two such values is a v_cndmask on registers (not a load from the kernel
// arguments, and no extra moves for the scalar-operand limit).
__device__ __forceinline__ float in_vgpr(float x)
{
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

__device__ __forceinline__ double in_vgpr(double x)
{
    double v;
    asm volatile("v_mov_b64 %0, %1" : "=v"(v) : "s"(x));
    return v;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Steps left before max_steps for the wave's most advanced lane that holds a trajectory, as a
// wave-uniform value (such a lane has at most max_steps steps: a lane reaching it is censored).
// At the start of a chunk it bounds every lane's count inside the chunk (all lanes step
// together), so whether a group can reach max_steps is one scalar comparison per group.
__device__ __forceinline__ uint32_t wave_steps_left(bool has, uint32_t n, uint32_t max_steps)
{
    uint32_t v = has ? n : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return max_steps - __builtin_amdgcn_readfirstlane(v);
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

// Where retired trajectories go: per-trajectory outputs (any may be NULL),
// the histogram layout and the block's LDS accumulators.
struct RetireTo {
    double *d_N, *d_lnw;
    uint32_t *d_steps;
    unsigned long long *cnt;
    double *sum;
    int nb;
    HistSpec hist;
};

// Retire one finished trajectory: per-trajectory outputs and LDS histogram.
__device__ __forceinline__ void retire(const RetireTo &t, uint64_t rel, uint32_t status, uint32_t n_steps, double N,
                                       double lnw)
{
    if (t.d_N) t.d_N[rel] = N;
    if (t.d_lnw) t.d_lnw[rel] = lnw;
    if (t.d_steps) t.d_steps[rel] = n_steps | status;
    if (status & kFlagCensored) {
        atomicAdd(&t.cnt[t.nb + 0], 1ull);
    } else if (status & kFlagEndedEarly) {
        atomicAdd(&t.cnt[t.nb + 1], 1ull);
    } else {
        const int b = bin_of(t.hist, N - t.hist.N_ref);
        const double w = exp(lnw);
        atomicAdd(&t.cnt[b], 1ull);
        atomicAdd(&t.sum[b], w);
        atomicAdd(&t.sum[t.nb + b], w * w);
        atomicAdd(&t.sum[2 * t.nb + b], lnw);
        atomicAdd(&t.sum[3 * t.nb + b], lnw * lnw);
        double *tot = t.sum + 4 * t.nb;
        atomicAdd(&tot[0], w);
        atomicAdd(&tot[1], w * w);
        atomicAdd(&tot[2], w * N);
        atomicAdd(&tot[3], w * N * N);
    }
    atomicAdd(&t.cnt[t.nb + 2], (unsigned long long)n_steps);
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

// V'/V for both potentials as 1/d, d = kx phi + s with s chosen per side:
//   piecewise linear  kx = 1, s = -c_+ (phi >= phi_T) or -c_- (phi < phi_T), c_+- = phi_T - V0/A_+-
//   exponential       kx = 0, s = 1/A_+ on both sides
// (no cancellation: d = phi - c is a single rounding).
struct DriftConsts {
    double kx, s_plus, s_minus;
};

__device__ __forceinline__ DriftConsts drift_consts(const Inst &I)
{
    DriftConsts k;
    if (I.pot_kind == kPotExponential) {
        k.kx = 0.0;
        k.s_plus = k.s_minus = 1.0 / I.A_plus;
    } else {
        k.kx = 1.0;
        k.s_plus = -(I.phi_T - I.V0 / I.A_plus);
        k.s_minus = -(I.phi_T - I.V0 / I.A_minus);
    }
    return k;
}

// V'/V of the Gaussian bump, eq. (potential_swagat), as one fraction:
//   2 m^2/(phi (m^2 + phi^2)) - x g/(Sigma (1 + g)),  x = (phi - phi_0)/Sigma,  g = K e^(-x^2/2).
// In ultra-slow roll the two terms nearly cancel; the single division keeps that to one rounding
// of the numerator's difference.
struct BumpConsts {
    double phi0, m2, two_m2, inv_sig, sig, K;
};

__device__ __forceinline__ BumpConsts bump_consts(const Inst &I)
{
    return BumpConsts{I.phi_T, I.bump_m2, 2.0 * I.bump_m2, 1.0 / I.bump_Sigma, I.bump_Sigma, I.bump_K};
}

__device__ __forceinline__ double bump_dlnV(const BumpConsts &b, double phi)
{
    const double x = (phi - b.phi0) * b.inv_sig;
    const double g = b.K * exp(-0.5 * x * x);
    const double d1 = phi * fma(phi, phi, b.m2);
    const double d2 = b.sig * (1.0 + g);
    // the quotient as the hardware reciprocal of the denominator (a normal number here: phi > 0
    // away from 0, Sigma (1 + g) > 0) with one Newton step, times the numerator: about 2e-15
    // relative, where the IEEE division would spend twice the instructions on the last ulp
    const double den = d1 * d2;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    return (b.two_m2 * d2 - x * g * d1) * r;
}

// The table size used by the kernels: a single node (constant noise) is
// staged as two equal nodes so one lookup serves every table.
__device__ __forceinline__ int staged_nodes(const Inst &I) { return I.n_tab > 1 ? I.n_tab : 2; }

// FP64 staging: the noise nodes, then the Box-Muller tables right after them.
__device__ __forceinline__ void stage_table64(const Inst &I, double2 *l_tab)
{
    const int n = staged_nodes(I);
    for (int i = threadIdx.x; i < n; i += blockDim.x) l_tab[i] = I.tab64[I.n_tab > 1 ? i : 0];
    stage_bm(l_tab + n);
}

// FP32 staging: the noise nodes, then the V'/V intervals right after them,
// scaled by half the time step (the step uses (V'/V) dN/2); all NaN for a
// single-node table, so that V'/V is computed exactly there.
__device__ __forceinline__ void stage_table32(const Inst &I, float4 *l_tab, float dN)
{
    const int n = staged_nodes(I);
    for (int i = threadIdx.x; i < n; i += blockDim.x) l_tab[i] = I.tab32[I.n_tab > 1 ? i : 0];
    float2 *l_r = reinterpret_cast<float2 *>(l_tab + n);
    const float nan = __builtin_nanf("");
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        float2 r = make_float2(nan, nan);
        if (I.n_tab > 1) {
            r = I.rtab32[i];
            r.x *= 0.5f * dN;
            r.y *= 0.5f * dN;
        }
        l_r[i] = r;
    }
}

// ---------------------------------------------------------------------------
// Learned control, tabulated: the amplitude a(phi, pi) is the bilinear
// interpolation of the network's values on a uniform grid of the normalised
// inputs (x0, x1) = ((phi - c0)/s0, (ln max(|pi|, 1e-30) - c1)/s1), clamped to
// the edge cells.  A deterministic function of the state is an admissible
// importance-sampling control (Sec. 4.1: the bias may depend on the state as
// long as the weight uses the same bias), and the weights below use this same
// amplitude, so the estimator stays unbiased.
//
// Replay (gradient) mode: the lanes integrate listed trajectories again with
// the same control and scatter each step's factor -xi sqrt(dN) (the on-policy
// value of -(e_k - a_k dN), e_k = a_k dN + xi_k sqrt(dN)) onto the four nodes
// of the step's cell with the bilinear weights, scaled by the path's w^2.  A
// lane keeps running sums for its current cell in registers and adds them to
// the block's LDS node array when the path leaves the cell or ends.
// ---------------------------------------------------------------------------
struct GridConsts64 {
    double k0, off0, k1, off1, imax0, imax1;
    int n1c;                   // cells per row, n1 - 1
};

__device__ __forceinline__ GridConsts64 grid_consts64(const Inst &I)
{
    GridConsts64 g;
    g.k0 = I.g_k0;
    g.off0 = I.g_off0;
    g.k1 = I.g_k1;
    g.off1 = I.g_off1;
    g.imax0 = (double)(I.g_n0 - 2);
    g.imax1 = (double)(I.g_n1 - 2);
    g.n1c = I.g_n1 - 1;
    return g;
}

// a(phi, pi) from the staged cells; also the cell and the fractions inside it.
// fmin/fmax map NaN and infinite coordinates onto the edge cells, so the cell
// index stays inside the table for any state.
__device__ __forceinline__ double grid_amp64(const GridConsts64 &g, const double2 *l_grid, double phi, double pi_,
                                             int &cell, double &f0, double &f1)
{
    const double u0 = fma(phi, g.k0, g.off0);
    const double u1 = fma(log(fmax(fabs(pi_), 1e-30)), g.k1, g.off1);
    const double i0 = fmin(fmax(floor(u0), 0.0), g.imax0);
    const double i1 = fmin(fmax(floor(u1), 0.0), g.imax1);
    f0 = fmin(fmax(u0 - i0, 0.0), 1.0);
    f1 = fmin(fmax(u1 - i1, 0.0), 1.0);
    cell = (int)i0 * g.n1c + (int)i1;
    const double2 c0 = l_grid[2 * cell], c1 = l_grid[2 * cell + 1];
    const double b0 = fma(f0, c0.y - c0.x, c0.x);
    const double b1 = fma(f0, c1.y - c1.x, c1.x);
    return fma(f1, b1 - b0, b0);
}

struct GridConsts32 {
    float k0, off0;            // u0 = x k0 + off0 with x = phi - phi_end
    float k1, off1;            // u1 = log2 max(|pi|, 1e-30) k1 + off1
    float imax0, imax1;
    int n1c;
};

__device__ __forceinline__ GridConsts32 grid_consts32(const Inst &I)
{
    GridConsts32 g;
    g.k0 = (float)I.g_k0;
    g.off0 = (float)fma(I.phi_end, I.g_k0, I.g_off0);
    g.k1 = (float)(I.g_k1 * 0.69314718055994531);
    g.off1 = (float)I.g_off1;
    g.imax0 = (float)(I.g_n0 - 2);
    g.imax1 = (float)(I.g_n1 - 2);
    g.n1c = I.g_n1 - 1;
    return g;
}

__device__ __forceinline__ float grid_amp32(const GridConsts32 &g, const float4 *l_grid, float x, float pi_, int &cell,
                                            float &f0, float &f1)
{
    const float u0 = fmaf(x, g.k0, g.off0);
    const float u1 = fmaf(__builtin_amdgcn_logf(fmaxf(fabsf(pi_), 1e-30f)), g.k1, g.off1);
    // clamps as one three-operand median each (both coordinates are finite)
    const float i0 = __builtin_amdgcn_fmed3f(floorf(u0), 0.0f, g.imax0);
    const float i1 = __builtin_amdgcn_fmed3f(floorf(u1), 0.0f, g.imax1);
    f0 = __builtin_amdgcn_fmed3f(u0 - i0, 0.0f, 1.0f);
    f1 = __builtin_amdgcn_fmed3f(u1 - i1, 0.0f, 1.0f);
    cell = (int)i0 * g.n1c + (int)i1;
    const float4 c = l_grid[cell];
    const float b0 = fmaf(f0, c.y - c.x, c.x);
    const float b1 = fmaf(f0, c.w - c.z, c.z);
    return fmaf(f1, b1 - b0, b0);
}

// Where a replay sends its results.
struct ReplayTo {
    const TailEntry *tail;
    double *l_G;                       // node weights of the block (LDS), n0 n1
    unsigned long long *mismatch;      // global count of replays that did not end with a passage
};

// Add a lane's running sums for `cell` (corner order (i0, i1), (i0 + 1, i1),
// (i0, i1 + 1), (i0 + 1, i1 + 1)) times ww to the LDS node weights.
template <typename T>
__device__ __forceinline__ void grad_flush(const ReplayTo &rp, int n1c, int cell, T s[4], double ww)
{
    if (cell >= 0) {
        const int k = cell + cell / n1c;          // node (i0, i1)
        const int n1 = n1c + 1;
        atomicAdd(&rp.l_G[k], ww * (double)s[0]);
        atomicAdd(&rp.l_G[k + n1], ww * (double)s[1]);
        atomicAdd(&rp.l_G[k + 1], ww * (double)s[2]);
        atomicAdd(&rp.l_G[k + n1 + 1], ww * (double)s[3]);
    }
    s[0] = s[1] = s[2] = s[3] = T(0);
}

template <typename T>
__device__ __forceinline__ void grad_add(T s[4], T c, T f0, T f1)
{
    const T p1 = c * f1, p0 = c - p1;        // c f1, c (1 - f1)
    s[0] += p0 - p0 * f0;
    s[1] += p0 * f0;
    s[2] += p1 - p1 * f0;
    s[3] += p1 * f0;
}

// ---------------------------------------------------------------------------
// Learned control, exact: output 0 of the 2 -> 64 -> 64 -> 2 tanh network itself at the
// normalised state (x0, x1), evaluated every mlp_every steps and held in between (the bias may be
// any deterministic function of the path's past states; the weights use the same amplitude, so
// the estimator stays unbiased).  Both evaluations take the network's sums in their own order.
//
// FP64 state: the parameters are staged in LDS as doubles, W2 transposed (word j 64 + i holds
// W2[i][j]), then W1, b1, b2, row 0 of W3 and b3[0]; the second layer is accumulated eight units
// at a time, each pass recomputing the 64 first-layer activations, so that a lane holds eight
// accumulators instead of 64 activations.
//
// FP32 state: the parameters are read in place from global memory through the constant address
// space.  Every lane of a wave reads the same word, so the loads become scalar loads and the
// multiply-adds take the weights as scalar operands (no LDS traffic); a lane keeps its 64
// first-layer activations in registers.  tanh s = 1 - 2/(e^(2s) + 1) from the hardware exp2 and
// reciprocal, exactly +-1 for large |s|.
// ---------------------------------------------------------------------------
constexpr int kMlpChunk = 8;
constexpr int kMlpLdsWords = kMlpHidden * kMlpHidden + 2 * kMlpHidden + 3 * kMlpHidden + 1;
constexpr size_t kMlpLdsBytes64 = ((size_t)kMlpLdsWords * 8 + 15) / 16 * 16;

__device__ __forceinline__ void stage_mlp64(const float *params, double *l_w)
{
    constexpr int H = kMlpHidden;
    for (int k = threadIdx.x; k < kMlpLdsWords; k += blockDim.x) {
        int src;
        if (k < H * H) {
            src = kOffW2 + (k % H) * H + k / H;       // word j H + i <- W2[i][j]
        } else {
            const int r = k - H * H;
            src = r < 2 * H ? kOffW1 + r                      // W1 [64][2]
                : r < 3 * H ? kOffB1 + (r - 2 * H)            // b1
                : r < 4 * H ? kOffB2 + (r - 3 * H)            // b2
                : r < 5 * H ? kOffW3 + (r - 4 * H)            // W3 row 0
                            : kOffB3;                         // b3[0]
        }
        l_w[k] = (double)params[src];
    }
}

__device__ __forceinline__ double mlp_out0_64(const double *l_w, double x0, double x1)
{
    constexpr int H = kMlpHidden;
    const double *W2t = l_w, *W1 = l_w + H * H, *b1 = W1 + 2 * H, *b2 = b1 + H, *W3 = b2 + H;
    double out = W3[H];
    for (int c = 0; c < H; c += kMlpChunk) {
        double acc[kMlpChunk];
#pragma unroll
        for (int i = 0; i < kMlpChunk; ++i) acc[i] = b2[c + i];
        for (int j = 0; j < H; ++j) {
            const double h = tanh(fma(W1[2 * j], x0, fma(W1[2 * j + 1], x1, b1[j])));
#pragma unroll
            for (int i = 0; i < kMlpChunk; ++i) acc[i] = fma(W2t[j * H + c + i], h, acc[i]);
        }
#pragma unroll
        for (int i = 0; i < kMlpChunk; ++i) out = fma(W3[c + i], tanh(acc[i]), out);
    }
    return out;
}

typedef __attribute__((address_space(4))) const float const_float;

// z[j] by a run-time index, as selects (folded away where j is a constant)
template <typename T>
__device__ __forceinline__ T pick4(const T z[4], int j)
{
    return j == 0 ? z[0] : j == 1 ? z[1] : j == 2 ? z[2] : z[3];
}

__device__ __forceinline__ float mlp_tanh32(float s)
{
    const float e = __builtin_amdgcn_exp2f(s * 2.8853900817779268f);   // e^(2s) = 2^(2 s log2 e)
    return fmaf(-2.0f, __builtin_amdgcn_rcpf(e + 1.0f), 1.0f);
}

__device__ __forceinline__ float mlp_out0_32(const_float *p, float x0, float x1)
{
    constexpr int H = kMlpHidden;
    float h[H];
#pragma unroll
    for (int j = 0; j < H; ++j)
        h[j] = mlp_tanh32(fmaf(p[kOffW1 + 2 * j], x0, fmaf(p[kOffW1 + 2 * j + 1], x1, p[kOffB1 + j])));
    float out = p[kOffB3];
    for (int o = 0; o < H; ++o) {
        const_float *row = p + kOffW2 + o * H;
        // two partial sums: two independent chains of multiply-adds
        float s0 = p[kOffB2 + o], s1 = 0.0f;
#pragma unroll
        for (int j = 0; j < H; j += 2) {
            s0 = fmaf(row[j], h[j], s0);
            s1 = fmaf(row[j + 1], h[j + 1], s1);
        }
        out = fmaf(p[kOffW3 + o], mlp_tanh32(s0 + s1), out);
    }
    return out;
}

// The network's normalised inputs: x0 = phi m_k0 + m_off0, x1 = ln max(|pi|, 1e-30) m_k1 + m_off1;
// FP32 state reads phi as x = phi - phi_end and takes log2.
struct NetConsts32 {
    float k0, off0, k1, off1;
};

__device__ __forceinline__ NetConsts32 net_consts32(const Inst &I)
{
    NetConsts32 q;
    q.k0 = (float)I.m_k0;
    q.off0 = (float)fma(I.phi_end, I.m_k0, I.m_off0);
    q.k1 = (float)(I.m_k1 * 0.69314718055994531);
    q.off1 = (float)I.m_off1;
    return q;
}

// ---------------------------------------------------------------------------
// FP64 state: the lanes of one wave integrate trajectories of instance I,
// claimed from `cursor` (global or LDS), until the range is exhausted.
//
// Steps are taken in groups of four (one Philox call).  Inside a group every
// lane computes every step; a lane whose trajectory ended earlier in the chunk
// keeps integrating a discarded state until the chunk ends and it is refilled,
// which keeps the group free of per-step exec-mask bookkeeping.  The end of a
// trajectory (first passage, eps_1 >= 1) is recorded in a branch that is taken
// about once per 1e4-1e5 steps and retired once the group is done.  Censoring
// at max_steps needs a test before every step, so groups that can reach
// max_steps take a separate variant; which groups can is decided once per chunk
// from the wave's largest step count (wave_steps_left).  GRAD: replay the trajectories listed in
// rp.tail (cursor over the list) and scatter the gradient factors instead of
// retiring into the histogram.
// ---------------------------------------------------------------------------
// TAB: 0 a single node (constant noise); 1 nodes in phi; 2 nodes in the run's time n dN (the
// table's phi_lo and inv_h then refer to N).
template <int BIAS, int TAB, bool ALLPOS, bool GRAD, int POT = kPotPiecewiseLinear>
__device__ __forceinline__ void lanes_fp64(const Inst &I, const RunArgs &R, const double2 *l_tab, const double2 *l_grid,
                                           const RetireTo &rt, const ReplayTo &rp, unsigned long long *cursor,
                                           uint64_t n_traj, uint64_t traj_offset)
{
    static_assert(!GRAD || BIAS == kBiasMlp, "replay needs the tabulated control");
    constexpr bool LEARNED = BIAS == kBiasMlp || BIAS == kBiasMlpExact;
    const double *l_w = reinterpret_cast<const double *>(l_grid);
    const uint32_t every = (uint32_t)I.mlp_every;
    // POT: kPotPiecewiseLinear serves both linear-family potentials (V'/V = 1/d below);
    // kPotGaussianBump computes the bump's V'/V
    const DriftConsts dk = drift_consts(I);
    const BumpConsts bc = bump_consts(I);
    const GridConsts64 gc = grid_consts64(I);
    const double S0 = l_tab[0].x, t0 = l_tab[0].y;
    const double2 *l_bm = l_tab + staged_nodes(I);
    const double dN = R.dN, sqrt_dN = R.sqrt_dN, phi_end = I.phi_end, phi_T = I.phi_T;
    const double a_const = (BIAS == kBiasConst) ? I.A : 0.0;
    const double half_a2_dN = 0.5 * a_const * a_const * dN;
    const double half_dN = 0.5 * dN;
    const double jmax = (double)(staged_nodes(I) - 2);
    const double s_plus = in_vgpr(dk.s_plus), s_minus = in_vgpr(dk.s_minus);

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, cursor, n_traj, exhausted);
    bool live = has;          // has a trajectory that has not ended yet
    double phi = I.phi_in, pi_ = I.pi_in, lnw = 0.0;
    uint32_t n = 0;
    double a_held = 0.0;      // exact network: its output at the last evaluation
    uint32_t next_eval = 0;   // exact network: the step of the next evaluation
    uint64_t traj = 0;        // GRAD: the listed trajectory
    double ww = 0.0;          // GRAD: its weight w^2
    int g_cell = -1;          // GRAD: cell of the running sums
    double g_s[4] = {0.0, 0.0, 0.0, 0.0};
    if (GRAD && has) {
        traj = rp.tail[rel].traj;
        ww = rp.tail[rel].ww;
    }
    PhiloxPre pre = philox_pre(GRAD ? traj : traj_offset + rel, I.instance, R.key0, R.key1);

    auto group = [&](auto censor_tag, const double z[4]) {
        constexpr bool CENSOR = decltype(censor_tag)::value;
        bool fresh = false;
        uint32_t ev_status, ev_n;   // written before use: read only where fresh is set
        double ev_N, ev_lnw;
#pragma unroll(BIAS == kBiasMlpExact ? 1 : 4)   // the exact network: one copy of its code
        for (int j = 0; j < 4; ++j) {
            if (CENSOR && live && n == I.max_steps) {
                ev_status = kFlagCensored;
                ev_n = n;
                ev_N = __builtin_nan("");
                ev_lnw = lnw;
                live = false;
                fresh = true;
            }
            double r;   // V'/V
            if (POT == kPotGaussianBump) {
                r = bump_dlnV(bc, phi);
            } else {
                // the hardware reciprocal (relative error below 5e-8) and one Newton step: 2.2e-15
                const double d = fma(phi, dk.kx, (phi >= phi_T) ? s_plus : s_minus);
                r = __builtin_amdgcn_rcp(d);
                r = fma(r, fma(-d, r, 1.0), r);
            }
            double S, t;
            if (TAB) {
                const double x = ((TAB == 2 ? (double)n * dN : phi) - I.phi_lo) * I.inv_h;
                const double jf = fmin(fmax(floor(x), 0.0), jmax);
                const double f = fmin(fmax(x - jf, 0.0), 1.0);
                const int jj = (int)jf;
                const double2 lo = l_tab[jj], hi = l_tab[jj + 1];
                S = lo.x + f * (hi.x - lo.x);
                t = lo.y + f * (hi.y - lo.y);
            } else {
                S = S0;
                t = t0;
            }
            double a = a_const;
            int cell = 0;
            double f0 = 0.0, f1 = 0.0;
            if (BIAS == kBiasMlp) a = grid_amp64(gc, l_grid, phi, pi_, cell, f0, f1);
            if (BIAS == kBiasMlpExact) {
                if (n == next_eval) {
                    a_held = mlp_out0_64(l_w, fma(phi, I.m_k0, I.m_off0),
                                         fma(log(fmax(fabs(pi_), 1e-30)), I.m_k1, I.m_off1));
                    next_eval += every;
                }
                a = a_held;
            }
            const double zs = pick4(z, j);                // xi sqrt(dN)
            const double noise = S * zs;
            // without a bias the amplitude is a literal 0, which IEEE arithmetic does not fold away:
            // the terms are left out instead (the same values, up to the sign of a zero)
            const double aS = a * S;
            const double phi_n = (BIAS == kBiasNone) ? phi + pi_ * dN + noise : phi + (pi_ + aS) * dN + noise;
            const double drift_pi = pi_ - (3.0 - 0.5 * pi_ * pi_) * (pi_ + r) * dN;
            const double pi_n = (BIAS == kBiasNone) ? drift_pi + t * noise : drift_pi + t * (aS * dN + noise);
            if (BIAS == kBiasConst) {
                if (ALLPOS) {
                    lnw -= a * zs + half_a2_dN;
                } else {
                    lnw -= (S > 0.0) ? a * zs + half_a2_dN : 0.0;
                }
            } else if (LEARNED) {
                const double dA = fma(a, zs, a * a * half_dN);
                lnw -= (ALLPOS || S > 0.0) ? dA : 0.0;
            }
            if (GRAD && live) {
                if (cell != g_cell) {
                    grad_flush(rp, gc.n1c, g_cell, g_s, ww);
                    g_cell = cell;
                }
                grad_add(g_s, (ALLPOS || S > 0.0) ? -zs : 0.0, f0, f1);
            }
            const bool crossed = phi_n <= phi_end;
            const bool ended = 0.5 * pi_n * pi_n >= 1.0;
            if (live && (crossed || ended)) {
                ev_status = crossed ? 0u : kFlagEndedEarly;
                ev_n = n + 1;
                ev_N = crossed ? (double)n * dN + dN * ((phi - phi_end) / (phi - phi_n)) : (double)(n + 1) * dN;
                ev_lnw = lnw;
                live = false;
                fresh = true;
            }
            phi = phi_n;
            pi_ = pi_n;
            n += 1;
        }
        if (fresh) {
            if (GRAD) {
                grad_flush(rp, gc.n1c, g_cell, g_s, ww);
                g_cell = -1;
                if (ev_status != 0u) atomicAdd(rp.mismatch, 1ull);
            } else {
                retire(rt, rel, ev_status, ev_n, ev_N, ev_lnw);
            }
        }
    };

    while (__any(has)) {
        const uint32_t left = wave_steps_left(has, n, I.max_steps);
        for (int k = 0; k < R.chunk; k += 4) {
            if (!__any(live)) break;
            uint32_t w[4];
            philox_call(n >> 2, pre, R.key0, R.key1, w);
            double z[4];
            box_muller64(w[0], w[1], sqrt_dN, l_bm, z[0], z[1]);
            box_muller64(w[2], w[3], sqrt_dN, l_bm, z[2], z[3]);
            if ((uint32_t)k + 4 > left) group(std::integral_constant<bool, true>(), z);
            else group(std::integral_constant<bool, false>(), z);
        }
        if (!live) has = false;
        if (claim(!has, rel, cursor, n_traj, exhausted)) {
            has = true;
            live = true;
            phi = I.phi_in;
            pi_ = I.pi_in;
            lnw = 0.0;
            n = 0;
            a_held = 0.0;
            next_eval = 0;
            if (GRAD) {
                traj = rp.tail[rel].traj;
                ww = rp.tail[rel].ww;
            }
            pre = philox_pre(GRAD ? traj : traj_offset + rel, I.instance, R.key0, R.key1);
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 state: x = phi - phi_end and pi each as an unevaluated pair of floats
// hi + lo.  A step adds its increment to the low word only (lo += dx) and
// reads the state as the rounded sum hi + lo; once per step group (16 steps, 4
// where the network is evaluated in the step) the pair is renormalised (Fast2Sum
// of hi and lo).
// Against an exact two-sum per step this leaves one rounding of the low word per
// step, at the scale of ulp(16 increments), far below the FP32 resolution of the
// state itself.
// ---------------------------------------------------------------------------
struct F32Consts {
    float xT_hi, xT_lo;        // phi_T - phi_end as a float pair
    float kx, s_plus, s_minus; // (V'/V) dN/2 = 1/(kx (phi - phi_T) + s), s = s_plus (phi >= phi_T) or s_minus
    float u_off;               // (phi_end - phi_lo) * inv_h: table coordinate of x = 0
    float inv_h;
    float t_scale, t_off;      // time tables: coordinate n dN inv_h - N_lo inv_h
    float jtop;                // n_tab - 1: the last record (slope 0, V'/V interval NaN)
    float dN, half_dN;
    float m2ln2_dN;            // -2 ln 2 dN: rho = sqrt(log2(u) m2ln2_dN) = sqrt(-2 ln u) sqrt(dN)
    float adN;                 // constant bias: A dN, the shift carried by each step's normal
};

__device__ __forceinline__ F32Consts f32_consts(const Inst &I, const RunArgs &R)
{
    F32Consts c;
    const double xT = I.phi_T - I.phi_end;
    c.xT_hi = (float)xT;
    c.xT_lo = (float)(xT - (double)c.xT_hi);
    const double two_over_dN = 2.0 / R.dN;
    if (I.pot_kind == kPotExponential) {
        c.kx = 0.0f;
        c.s_plus = c.s_minus = (float)(two_over_dN / I.A_plus);
    } else {
        c.kx = (float)two_over_dN;
        c.s_plus = (float)(I.V0 / I.A_plus * two_over_dN);
        c.s_minus = (float)(I.V0 / I.A_minus * two_over_dN);
    }
    c.u_off = (float)((I.phi_end - I.phi_lo) * I.inv_h);
    c.inv_h = (float)I.inv_h;
    c.t_scale = (float)(R.dN * I.inv_h);
    c.t_off = (float)(-I.phi_lo * I.inv_h);
    c.jtop = (float)(staged_nodes(I) - 1);
    c.dN = (float)R.dN;
    c.half_dN = (float)(0.5 * R.dN);
    c.m2ln2_dN = (float)(-2.0 * 0.69314718055994531 * R.dN);
    c.adN = (I.bias_kind == kBiasConst) ? (float)(I.A * R.dN) : 0.0f;
    return c;
}

// Box-Muller in FP32 on uniforms fl32(w) 2^-32 + 2^-33: the same uniform as the
// FP64 path, rounded to 24 significant bits (relative, not absolute, resolution,
// so the radius stays accurate for small u).  Never 0; at most 1.0f, where
// log2 gives 0 and the radius -0 or 0.  v_log_f32 returns log2, v_sin_f32 /
// v_cos_f32 take turns.  Returns xi sqrt(dN) + off for the two steps of the pair.
__device__ __forceinline__ void box_muller32(uint32_t wa, uint32_t wb, float m2ln2_dN, float off, float &za, float &zb)
{
    const float ua = fmaf((float)wa, 0x1p-32f, 0x1p-33f);
    const float ub = fmaf((float)wb, 0x1p-32f, 0x1p-33f);
    const float rho = __builtin_amdgcn_sqrtf(__builtin_amdgcn_logf(ua) * m2ln2_dN);
    za = fmaf(rho, __builtin_amdgcn_cosf(ub), off);
    zb = fmaf(rho, __builtin_amdgcn_sinf(ub), off);
}

template <int BIAS, int TAB, bool ALLPOS, bool GRAD>
__device__ __forceinline__ void lanes_fp32(const Inst &I, const RunArgs &R, const float4 *l_tab, const float4 *l_grid,
                                           const RetireTo &rt, const ReplayTo &rp, unsigned long long *cursor,
                                           uint64_t n_traj, uint64_t traj_offset)
{
    static_assert(!GRAD || BIAS == kBiasMlp, "replay needs the tabulated control");
    constexpr bool LEARNED = BIAS == kBiasMlp || BIAS == kBiasMlpExact;
    // steps per group: 16 (four generator calls), so that the group's fixed work (table record,
    // renormalisation, FP64 sums, loop control) is shared by 16 steps; the normals of the whole
    // group are formed first.  The exact network keeps groups of 4 and one copy of its code.
    constexpr int G = (BIAS == kBiasMlpExact) ? 4 : 16;
    const_float *wp = (const_float *)(uintptr_t)I.mlp_params;
    const NetConsts32 nq = net_consts32(I);
    const uint32_t every = (uint32_t)I.mlp_every;
    const F32Consts c = f32_consts(I, R);
    const GridConsts32 gc = grid_consts32(I);
    const float S0 = l_tab[0].x, t0 = l_tab[0].z;
    const float2 *l_rtab = reinterpret_cast<const float2 *>(l_tab + staged_nodes(I));
    const double x_in = I.phi_in - I.phi_end;
    const float x_in_hi = (float)x_in, x_in_lo = (float)(x_in - (double)x_in_hi);
    const float pi_in_hi = (float)I.pi_in, pi_in_lo = (float)(I.pi_in - (double)pi_in_hi);
    const double dN = R.dN;
    const double A = (BIAS == kBiasConst) ? I.A : 0.0;
    const double half_a2_dN = 0.5 * A * A * dN;
    const float s_plus = in_vgpr(c.s_plus), s_minus = in_vgpr(c.s_minus);

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, cursor, n_traj, exhausted);
    bool live = has;          // has a trajectory that has not ended yet
    // state: x = xh + xl, pi = ph + pl; xs, ps their rounded sums (what a step reads; xs is formed
    // each step only where a step reads it, and otherwise once per group)
    float xh = x_in_hi, xl = x_in_lo, ph = pi_in_hi, pl = pi_in_lo;
    float xs = x_in_hi, ps = pi_in_hi;
    double zsum = 0.0;        // constant bias: sum of z = xi sqrt(dN) + a dN over steps with S > 0
    uint32_t n_on = 0;        // constant bias: number of such steps (counted only when some node has S = 0)
    double lnw = 0.0;         // learned bias: ln w up to the current group
    uint32_t n = 0;
    float a_held = 0.0f;      // exact network: its output at the last evaluation
    uint32_t next_eval = 0;   // exact network: the step of the next evaluation
    uint64_t traj = 0;        // GRAD: the listed trajectory
    double ww = 0.0;          // GRAD: its weight w^2
    int g_cell = -1;          // GRAD: cell of the running sums
    float g_s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (GRAD && has) {
        traj = rp.tail[rel].traj;
        ww = rp.tail[rel].ww;
    }
    PhiloxPre pre = philox_pre(GRAD ? traj : traj_offset + rel, I.instance, R.key0, R.key1);

    // constant bias: each step's normal carries the drift shift, z = xi sqrt(dN) + c.adN with
    // c.adN = fl32(A dN), so the exponent of eq. (weight_A) in 1D over k steps,
    // -A sum xi sqrt(dN) - k A^2 dN / 2, is -A sum z + k (A c.adN - A^2 dN / 2)
    const double lnw_step = A * (double)c.adN - half_a2_dN;
    auto lnw_of = [&](double zs_total, uint32_t steps_on) -> double {
        return (BIAS == kBiasNone) ? 0.0 : -A * zs_total + (double)steps_on * lnw_step;
    };

    // Phi tables: a lane whose interval at the group start holds an interpolated V'/V reads that
    // record once for the whole group, and each step evaluates S, tan theta and V'/V on that
    // interval's linear piece: value at x = xh plus slope per unit x times xl (x - xh = xl within
    // the group), the values and slopes formed once per group.  Inside the interval
    // this is the table's interpolation; where the group's path passes a node it extends the start
    // interval's piece instead of switching to the next one, which differs from the interpolation
    // by the change of slope at the node times the distance past it (second order in the node
    // spacing for a table of a smooth function).  A lane whose interval is NaN-marked (table
    // edges, the kink, tables that do not qualify) takes the record of each step's own clamped
    // coordinate instead.  The choice is the lane's own, so a trajectory's
    // arithmetic does not depend on the other lanes of its wave: SPAN groups, where no live lane is
    // in a NaN interval, run the first form only; the other groups run both and select per lane.
    // the group-start record's S, tan theta and V'/V at x = xh and their slopes per unit x
    float g_S = 0.0f, g_dS = 0.0f, g_t = 0.0f, g_dt = 0.0f, g_r = 0.0f, g_dr = 0.0f;

    // The epsilon_1 = 1 end (|pi| >= sqrt 2) in SPAN groups.  While |pi| < sqrt 2, a step changes pi
    // by at most delta = 6 (sqrt2 dN/2 + |V'/V| dN/2) + |tan theta| S |z| (|pi^2 - 6| <= 6), where
    // S, tan theta and V'/V are read from a smooth record extended past its interval by at most
    // the D intervals a group's path can move (|dx| <= sqrt2 dN + S |z|), and |z| <= 6.8 sqrt(dN) +
    // |a| dN (the Box-Muller radius is at most sqrt(66 ln 2 dN)).  A lane with |pi| <= pi_safe at
    // the group start therefore stays below sqrt 2 (1 - 1e-3) for 16 steps (5 % margin on delta),
    // and a SPAN group whose live lanes all qualify leaves the end test out; the other SPAN groups
    // keep it.  With no usable bound (fine grids, where D is large) pi_safe is -1: no lane
    // qualifies, and every group keeps the test.
    float pi_safe = -1.0f;
    if (TAB == 1 && !LEARNED) {
        const float zmax = fmaf(6.8f, __builtin_amdgcn_sqrtf(c.dN), fabsf((float)A) * c.dN);
        const float D = fmaf(16.0f * c.inv_h, fmaf(2.0f * I.rec_S, zmax, 1.4143f * c.dN), 1.0f);
        const float Sx = fmaf(I.rec_dS, D, I.rec_S);
        const float Tx = fmaf(I.rec_dt, D, I.rec_t);
        const float Rx = fmaf(I.rec_dr, D, I.rec_r) * c.half_dN;
        const float delta = fmaf(6.0f, fmaf(0.7072f, c.dN, Rx), Tx * Sx * zmax);
        if (Sx <= 2.0f * I.rec_S && delta == delta && delta >= 0.0f && delta < 1.0f)
            pi_safe = fmaf(-16.8f, delta, 1.4128f);
    }

    auto group = [&](auto censor_tag, auto span_tag, auto end_tag, const float z[G]) {
        constexpr bool CENSOR = decltype(censor_tag)::value;
        constexpr bool SPAN = decltype(span_tag)::value;
        constexpr bool END = decltype(end_tag)::value;   // test the eps_1 = 1 end in each step
        static_assert(!SPAN || (TAB == 1 && !CENSOR), "one record per group: phi tables, no censoring");
        // the rounded sum xs is read by a step only for a per-step table lookup and by the control
        constexpr bool STEP_XS = LEARNED || (TAB == 1 && !SPAN);
        float zacc = 0.0f;        // constant bias: sum of this group's xi sqrt(dN); learned: of its dA
        bool fresh = false;
        uint32_t ev_code;         // written before use: read only where fresh is set
        double ev_N, ev_lnw;
        auto lnw_now = [&](uint32_t steps) -> double {
            if (LEARNED) return lnw - (double)zacc;
            return lnw_of(zsum + (double)zacc, ALLPOS ? steps : n_on);
        };
#pragma unroll(BIAS == kBiasMlpExact ? 1 : G)   // the exact network: one copy of its code
        for (int j = 0; j < G; ++j) {
            const float zj = (G == 4) ? pick4(z, j) : z[j];
            if (CENSOR && live && n + j == I.max_steps) {
                ev_code = (n + j) | kFlagCensored;
                ev_N = __builtin_nan("");
                ev_lnw = lnw_now(n + j);
                live = false;
                fresh = true;
            }
            // (V'/V) dN/2 exactly: 1/(kx (phi - phi_T) + s), phi - phi_T = (xh - xT_hi) + (xl - xT_lo)
            auto drift_exact = [&]() -> float {
                const float dT = (xh - c.xT_hi) + (xl - c.xT_lo);
                return __builtin_amdgcn_rcpf(fmaf(dT, c.kx, (dT >= 0.0f) ? s_plus : s_minus));
            };
            float S, t, r;        // r = (V'/V) dN/2
            if (TAB == 2) {
                // time table: the node at n dN; V'/V exactly (the V'/V intervals follow phi)
                const float u = __builtin_amdgcn_fmed3f(fmaf((float)(n + j), c.t_scale, c.t_off), 0.0f, c.jtop);
                const float f = __builtin_amdgcn_fractf(u);
                const float4 node = l_tab[(int)u];
                S = fmaf(f, node.y, node.x);
                t = fmaf(f, node.w, node.z);
                r = drift_exact();
            } else if (SPAN) {
                S = fmaf(xl, g_dS, g_S);
                t = fmaf(xl, g_dt, g_t);
                r = fmaf(xl, g_dr, g_r);
            } else if (TAB) {
                // the coordinate clamped to [0, n_tab - 1]: its integer part is the record, its
                // fraction the weight; past the last node the last record (slope 0) gives the
                // edge value, and its NaN V'/V interval the exact V'/V
                const float u = __builtin_amdgcn_fmed3f(fmaf(xs, c.inv_h, c.u_off), 0.0f, c.jtop);
                const float f = __builtin_amdgcn_fractf(u);
                const float4 node = l_tab[(int)u];
                const float2 rn = l_rtab[(int)u];
                S = fmaf(f, node.y, node.x);
                t = fmaf(f, node.w, node.z);
                // V'/V interpolated in the interval (error below FP32 resolution); NaN marks the
                // intervals where it is computed exactly instead: the two edge intervals, which
                // also take every clamped coordinate outside the table, the two intervals at the
                // kink phi_T, and every interval of a table that does not qualify
                r = fmaf(f, rn.y, rn.x);
                if (TAB == 1 && g_r == g_r) {
                    // the lane's group-start interval is smooth: the arithmetic of a SPAN group
                    S = fmaf(xl, g_dS, g_S);
                    t = fmaf(xl, g_dt, g_t);
                    r = fmaf(xl, g_dr, g_r);
                }
                if (__any(r != r)) {
                    // a real branch (rarely taken): the volatile asm keeps the compiler from
                    // computing the exact value in every step and selecting
                    asm volatile("; exact V'/V");
                    if (r != r) r = drift_exact();
                }
            } else {
                S = S0;
                t = t0;
                r = drift_exact();
            }
            float a = 0.0f;       // the learned amplitude
            int cell = 0;
            float f0 = 0.0f, f1 = 0.0f;
            if (BIAS == kBiasMlp) a = grid_amp32(gc, l_grid, xs, ps, cell, f0, f1);
            if (BIAS == kBiasMlpExact) {
                if (n + j == next_eval) {
                    a_held = mlp_out0_32(wp, fmaf(xs, nq.k0, nq.off0),
                                         fmaf(__builtin_amdgcn_logf(fmaxf(fabsf(ps), 1e-30f)), nq.k1, nq.off1));
                    next_eval += every;
                }
                a = a_held;
            }
            // Bn = S (a dN + xi sqrt(dN)): the bias and noise increments of phi (a constant bias
            // rides in z = xi sqrt(dN) + a dN; the learned one is added here, z = xi sqrt(dN))
            const float Bn = S * (LEARNED ? fmaf(a, c.dN, zj) : zj);
            if (BIAS == kBiasConst) {
                if (ALLPOS) {
                    zacc = (j == 0) ? z[0] : zacc + zj;
                } else {
                    const bool on = S > 0.0f;
                    zacc += on ? zj : 0.0f;
                    n_on += on ? 1u : 0u;
                }
            } else if (LEARNED) {
                const float dA = fmaf(a, zj, a * a * (0.5f * c.dN));
                zacc += (ALLPOS || S > 0.0f) ? dA : 0.0f;
            }
            if (GRAD && live) {
                if (cell != g_cell) {
                    grad_flush(rp, gc.n1c, g_cell, g_s, ww);
                    g_cell = cell;
                }
                grad_add(g_s, (ALLPOS || S > 0.0f) ? -zj : 0.0f, f0, f1);
            }
            // x += pi dN + Bn; pi += (pi^2 - 6)(pi dN/2 + (V'/V) dN/2) + tan(theta) Bn, i.e.
            // -(3 - pi^2/2)(pi + V'/V) dN plus the bias and noise along (1, tan theta).  The pi
            // terms go into their low word by two FMAs; the x increment is formed first and added
            // once, since adding its two parts one at a time rounds twice at the low word's scale,
            // which shifted the crossing (the mean N by ~1e-6 against FP64 on the same normals).
            const float x0l = xl;
            xl += fmaf(ps, c.dN, Bn);
            pl = fmaf(fmaf(ps, ps, -6.0f), fmaf(ps, c.half_dN, r), fmaf(t, Bn, pl));
            if (STEP_XS) xs = xh + xl;
            ps = ph + pl;
            // x <= 0: the sign of a rounded sum is that of the exact one, so this is xs <= 0
            const bool crossed = xl <= -xh;
            // eps_1 = pi^2/2 >= 1: |pi| >= the float just above sqrt(2) (no float lies between
            // sqrt(2) and it, so this is pi^2 >= 2 for float pi); left out of the groups where no
            // live lane can get there (pi_safe above)
            const bool ended = END && fabsf(ps) >= 0x1.6a09e8p+0f;
            // live and fresh are updated outside the branch, so that they stay lane masks
            const bool hit = live && (crossed || ended);
            if (hit) {
                // both candidates, then a select on the crossing mask: no divergent branch inside.
                // The state passes through an empty volatile asm first, which keeps the compiler
                // from moving this rarely taken work in front of the branch (into every step).
                float bh = xh, b0 = x0l, b1 = xl;
                uint32_t nb = n + j;
                asm volatile("; passage event" : "+v"(bh), "+v"(b0), "+v"(b1), "+v"(nb));
                const double x0 = (double)bh + (double)b0;
                const double x1 = (double)bh + (double)b1;
                const double N_cross = (double)nb * dN + dN * (x0 / (x0 - x1));
                const double N_end = (double)(nb + 1) * dN;
                ev_code = (nb + 1) | (crossed ? 0u : kFlagEndedEarly);
                ev_N = crossed ? N_cross : N_end;
                ev_lnw = lnw_now(nb + 1);
            }
            live = live && !hit;
            fresh = fresh || hit;
        }
        n += G;
        if (LEARNED) lnw -= (double)zacc;
        else zsum += (double)zacc;
        if (fresh) {
            if (GRAD) {
                grad_flush(rp, gc.n1c, g_cell, g_s, ww);
                g_cell = -1;
                if ((ev_code & ~kStepMask) != 0u) atomicAdd(rp.mismatch, 1ull);
            } else {
                retire(rt, rel, ev_code & ~kStepMask, ev_code & kStepMask, ev_N, ev_lnw);
            }
        }
        // renormalise the pairs once per group (Fast2Sum of hi and the accumulated lo; ps, and xs
        // where a step reads it, are their rounded sums already)
        if (!STEP_XS) xs = xh + xl;
        xl = xl - (xs - xh);
        xh = xs;
        pl = pl - (ps - ph);
        ph = ps;
    };

    // n_hi: a wave-uniform upper bound on n over the lanes that hold a trajectory.  All lanes step
    // together and a refilled lane restarts at 0, so adding each chunk's steps keeps it a bound;
    // the exact maximum (a cross-lane reduction) is formed only once the bound comes within a
    // chunk of max_steps, so the groups that can reach max_steps are the same as with the exact
    // count at every chunk
    uint32_t n_hi = 0;
    while (__any(has)) {
        if ((uint64_t)n_hi + (uint64_t)R.chunk + G > I.max_steps)
            n_hi = I.max_steps - wave_steps_left(has, n, I.max_steps);
        const uint32_t left = I.max_steps - n_hi;
        int k = 0;
        for (; k < R.chunk; k += G) {
            if (!__any(live)) break;
            uint32_t w[G];
#pragma unroll
            for (int q = 0; q < G; q += 4) philox_call((n >> 2) + (uint32_t)(q >> 2), pre, R.key0, R.key1, w + q);
            float z[G];
            const float off = (BIAS == kBiasConst) ? c.adN : 0.0f;
#pragma unroll
            for (int q = 0; q < G; q += 2) box_muller32(w[q], w[q + 1], c.m2ln2_dN, off, z[q], z[q + 1]);
            using T = std::integral_constant<bool, true>;
            using F = std::integral_constant<bool, false>;
            if constexpr (TAB == 1) {
                // the record of the lane's interval at the group start
                const float u0 = __builtin_amdgcn_fmed3f(fmaf(xs, c.inv_h, c.u_off), 0.0f, c.jtop);
                const int j0 = (int)u0;
                const float4 g_node = l_tab[j0];
                const float2 g_rn = l_rtab[j0];
                const float fh = fmaf(xh, c.inv_h, c.u_off - (float)j0);   // the fraction at x = xh
                g_S = fmaf(fh, g_node.y, g_node.x);
                g_dS = g_node.y * c.inv_h;
                g_t = fmaf(fh, g_node.w, g_node.z);
                g_dt = g_node.w * c.inv_h;
                g_r = fmaf(fh, g_rn.y, g_rn.x);
                g_dr = g_rn.y * c.inv_h;
            }
            if ((uint32_t)k + G > left) {
                group(T(), F(), T(), z);
            } else {
                if constexpr (TAB == 1) {
                    if (__builtin_amdgcn_ballot_w64(live && g_r != g_r) != 0) {
                        group(F(), F(), T(), z);
                    } else if constexpr (LEARNED) {
                        group(F(), T(), T(), z);
                    } else {
                        if (__builtin_amdgcn_ballot_w64(live && fabsf(ps) > pi_safe) == 0)
                            group(F(), T(), F(), z);
                        else group(F(), T(), T(), z);
                    }
                } else {
                    group(F(), F(), T(), z);
                }
            }
        }
        n_hi += (uint32_t)k;
        if (!live) has = false;
        if (claim(!has, rel, cursor, n_traj, exhausted)) {
            has = true;
            live = true;
            xh = xs = x_in_hi;
            xl = x_in_lo;
            ph = ps = pi_in_hi;
            pl = pi_in_lo;
            zsum = 0.0;
            n_on = 0;
            lnw = 0.0;
            n = 0;
            a_held = 0.0f;
            next_eval = 0;
            if (GRAD) {
                traj = rp.tail[rel].traj;
                ww = rp.tail[rel].ww;
            }
            pre = philox_pre(GRAD ? traj : traj_offset + rel, I.instance, R.key0, R.key1);
        }
    }
}
// ---------------------------------------------------------------------------
// FP64 state with 2D noise (eq. full_langevin_equation): two normals per step,
// noise S (xi_1, xi_2) sqrt(dN) with S the interpolated symmetric square root of
// the covariance, bias B = a S e with e the interpolated principal axis, and
// dA = a e.xi sqrt(dN) + a^2 |e|^2 dN / 2, eq. (weight_A) for B = S (a e).  Step
// n takes call n >> 1 of the generator: (u0, u1) for step 2m, (u2, u3) for
// 2m + 1, so a group of two steps takes one call.  The structure (groups,
// event capture, claims) is that of lanes_fp64.
// ---------------------------------------------------------------------------
struct Node2d {
    double Spp, Spq, Sqq, e1, e2;
};

__device__ __forceinline__ Node2d lerp_node2d(const double2 *l_tab, int j, double f)
{
    const double2 a0 = l_tab[3 * j], a1 = l_tab[3 * j + 1], a2 = l_tab[3 * j + 2];
    const double2 b0 = l_tab[3 * j + 3], b1 = l_tab[3 * j + 4], b2 = l_tab[3 * j + 5];
    Node2d n;
    n.Spp = a0.x + f * (b0.x - a0.x);
    n.Spq = a0.y + f * (b0.y - a0.y);
    n.Sqq = a1.x + f * (b1.x - a1.x);
    n.e1 = a1.y + f * (b1.y - a1.y);
    n.e2 = a2.x + f * (b2.x - a2.x);
    return n;
}

template <int BIAS, bool ALLPOS, bool TIME>
__device__ __forceinline__ void lanes_fp64_2d(const Inst &I, const RunArgs &R, const double2 *l_tab,
                                              const RetireTo &rt, unsigned long long *cursor, uint64_t n_traj,
                                              uint64_t traj_offset)
{
    const DriftConsts dk = drift_consts(I);
    const double dN = R.dN, sqrt_dN = R.sqrt_dN, phi_end = I.phi_end, phi_T = I.phi_T;
    const double a = (BIAS == kBiasConst) ? I.A : 0.0;
    const double half_a2_dN = 0.5 * a * a * dN;
    const double jmax = (double)(staged_nodes(I) - 2);
    const double2 *l_bm = l_tab + 3 * staged_nodes(I);
    const double s_plus = in_vgpr(dk.s_plus), s_minus = in_vgpr(dk.s_minus);

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, cursor, n_traj, exhausted);
    bool live = has;
    double phi = I.phi_in, pi_ = I.pi_in, lnw = 0.0;
    uint32_t n = 0;
    PhiloxPre pre = philox_pre(traj_offset + rel, I.instance, R.key0, R.key1);

    // groups of two steps: one Philox call gives both steps' (xi_1, xi_2)
    auto group = [&](auto censor_tag, const double z[4]) {
        constexpr bool CENSOR = decltype(censor_tag)::value;
        bool fresh = false;
        uint32_t ev_status, ev_n;   // written before use: read only where fresh is set
        double ev_N, ev_lnw;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            if (CENSOR && live && n == I.max_steps) {
                ev_status = kFlagCensored;
                ev_n = n;
                ev_N = __builtin_nan("");
                ev_lnw = lnw;
                live = false;
                fresh = true;
            }
            const double d = fma(phi, dk.kx, (phi >= phi_T) ? s_plus : s_minus);
            double r = __builtin_amdgcn_rcp(d);          // V'/V: reciprocal and one Newton step
            r = fma(r, fma(-d, r, 1.0), r);
            // table coordinate: phi, or the run's time n dN for a time-indexed table
            const double x = ((TIME ? (double)n * dN : phi) - I.phi_lo) * I.inv_h;
            const double jf = fmin(fmax(floor(x), 0.0), jmax);
            const double f = fmin(fmax(x - jf, 0.0), 1.0);
            const Node2d S = lerp_node2d(l_tab, (int)jf, f);
            const double z1 = z[2 * j], z2 = z[2 * j + 1];          // xi sqrt(dN)
            const double noise_phi = S.Spp * z1 + S.Spq * z2;
            const double noise_pi = S.Spq * z1 + S.Sqq * z2;
            // without a bias the amplitude is a literal 0, which IEEE arithmetic does not fold away:
            // the terms are left out instead (the same values, up to the sign of a zero)
            const double B_phi = a * (S.Spp * S.e1 + S.Spq * S.e2);
            const double B_pi = a * (S.Spq * S.e1 + S.Sqq * S.e2);
            const double phi_n =
                (BIAS == kBiasNone) ? phi + pi_ * dN + noise_phi : phi + (pi_ + B_phi) * dN + noise_phi;
            const double drift_pi = pi_ - (3.0 - 0.5 * pi_ * pi_) * (pi_ + r) * dN;
            const double pi_n = (BIAS == kBiasNone) ? drift_pi + noise_pi : drift_pi + B_pi * dN + noise_pi;
            if (BIAS != kBiasNone) {
                const double dA = a * (S.e1 * z1 + S.e2 * z2) + half_a2_dN * (S.e1 * S.e1 + S.e2 * S.e2);
                if (ALLPOS) lnw -= dA;
                else lnw -= (S.Spp != 0.0 || S.Spq != 0.0 || S.Sqq != 0.0) ? dA : 0.0;
            }
            const bool crossed = phi_n <= phi_end;
            const bool ended = 0.5 * pi_n * pi_n >= 1.0;
            if (live && (crossed || ended)) {
                ev_status = crossed ? 0u : kFlagEndedEarly;
                ev_n = n + 1;
                ev_N = crossed ? (double)n * dN + dN * ((phi - phi_end) / (phi - phi_n)) : (double)(n + 1) * dN;
                ev_lnw = lnw;
                live = false;
                fresh = true;
            }
            phi = phi_n;
            pi_ = pi_n;
            n += 1;
        }
        if (fresh) retire(rt, rel, ev_status, ev_n, ev_N, ev_lnw);
    };

    while (__any(has)) {
        const uint32_t left = wave_steps_left(has, n, I.max_steps);
        for (int k = 0; k < R.chunk; k += 2) {
            if (!__any(live)) break;
            uint32_t w[4];
            philox_call(n >> 1, pre, R.key0, R.key1, w);
            double z[4];
            box_muller64(w[0], w[1], sqrt_dN, l_bm, z[0], z[1]);
            box_muller64(w[2], w[3], sqrt_dN, l_bm, z[2], z[3]);
            if ((uint32_t)k + 2 > left) group(std::integral_constant<bool, true>(), z);
            else group(std::integral_constant<bool, false>(), z);
        }
        if (!live) has = false;
        if (claim(!has, rel, cursor, n_traj, exhausted)) {
            has = true;
            live = true;
            phi = I.phi_in;
            pi_ = I.pi_in;
            lnw = 0.0;
            n = 0;
            pre = philox_pre(traj_offset + rel, I.instance, R.key0, R.key1);
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 state with 2D noise (eq. full_langevin_equation): the float-pair state of
// lanes_fp32 with the noise, bias and weight of lanes_fp64_2d.  Step n takes
// (xi_1, xi_2) from generator call n >> 1 as the FP64 2D path does ((u0, u1) for
// step 2m, (u2, u3) for step 2m + 1), so the two paths see the same numbers; a
// group of 16 steps takes eight calls.  Node record, three float4:
// (S_pp, slope, S_pq, slope), (S_qq, slope, e_phi, slope), (e_pi, slope, r, slope)
// with r = (V'/V) dN/2 interpolated in the interval, NaN where V'/V is computed
// exactly (as in the 1D FP32 table; all NaN on a time axis).  A constant bias
// B = a S e enters through shifted normals, B dN + S xi sqrt(dN) = S (xi sqrt(dN)
// + a dN e), and dA = a e.xi sqrt(dN) + a^2 |e|^2 dN/2 is summed per group in
// FP32 and across groups in FP64.
// ---------------------------------------------------------------------------
template <int BIAS, bool ALLPOS, bool TIME>
__device__ __forceinline__ void lanes_fp32_2d(const Inst &I, const RunArgs &R, const float4 *l_tab, const RetireTo &rt,
                                              unsigned long long *cursor, uint64_t n_traj, uint64_t traj_offset)
{
    // steps per group: 16 (eight generator calls, the normals of the whole group formed first)
    constexpr int G = 16;
    const F32Consts c = f32_consts(I, R);
    const double x_in = I.phi_in - I.phi_end;
    const float x_in_hi = (float)x_in, x_in_lo = (float)(x_in - (double)x_in_hi);
    const float pi_in_hi = (float)I.pi_in, pi_in_lo = (float)(I.pi_in - (double)pi_in_hi);
    const double dN = R.dN;
    const float a = (BIAS == kBiasConst) ? (float)I.A : 0.0f;
    const float adN = a * c.dN;                 // the normals' shift per unit of e
    const float half_a2_dN = 0.5f * a * a * c.dN;
    const float s_plus = in_vgpr(c.s_plus), s_minus = in_vgpr(c.s_minus);

    bool exhausted = false;
    uint64_t rel = 0;
    bool has = claim(true, rel, cursor, n_traj, exhausted);
    bool live = has;
    float xh = x_in_hi, xl = x_in_lo, ph = pi_in_hi, pl = pi_in_lo;
    float xs = x_in_hi, ps = pi_in_hi;          // xs is formed each step only for a per-step lookup
    double lnw = 0.0;
    uint32_t n = 0;
    PhiloxPre pre = philox_pre(traj_offset + rel, I.instance, R.key0, R.key1);

    // Phi tables: the lane's group-start record, as in lanes_fp32: each entry's value at x = xh
    // and its slope per unit x, so that a step of a lane whose start interval is smooth evaluates
    // every entry as value + slope * xl (the start interval's linear piece, extended past a node
    // the group's path passes); lanes in NaN-marked intervals read each step's own record.
    float g_v[6], g_d[6];           // S_pp, S_pq, S_qq, e_phi, e_pi, r
#pragma unroll
    for (int q = 0; q < 6; ++q) g_v[q] = g_d[q] = 0.0f;

    auto group = [&](auto censor_tag, auto span_tag, const float z[2 * G]) {
        constexpr bool CENSOR = decltype(censor_tag)::value;
        constexpr bool SPAN = decltype(span_tag)::value;
        static_assert(!SPAN || (!TIME && !CENSOR), "one record per group: phi tables, no censoring");
        constexpr bool STEP_XS = !TIME && !SPAN;
        float zacc = 0.0f;        // this group's sum of dA
        bool fresh = false;
        uint32_t ev_code;
        double ev_N, ev_lnw;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (CENSOR && live && n + j == I.max_steps) {
                ev_code = (n + j) | kFlagCensored;
                ev_N = __builtin_nan("");
                ev_lnw = lnw - (double)zacc;
                live = false;
                fresh = true;
            }
            float Spp, Spq, Sqq, e1, e2, r;     // r = (V'/V) dN/2
            if (SPAN) {
                Spp = fmaf(xl, g_d[0], g_v[0]);
                Spq = fmaf(xl, g_d[1], g_v[1]);
                Sqq = fmaf(xl, g_d[2], g_v[2]);
                e1 = fmaf(xl, g_d[3], g_v[3]);
                e2 = fmaf(xl, g_d[4], g_v[4]);
                r = fmaf(xl, g_d[5], g_v[5]);
            } else {
                const float u = __builtin_amdgcn_fmed3f(
                    TIME ? fmaf((float)(n + j), c.t_scale, c.t_off) : fmaf(xs, c.inv_h, c.u_off), 0.0f, c.jtop);
                const float f = __builtin_amdgcn_fractf(u);
                const float4 *rec = l_tab + 3 * (int)u;
                const float4 A0 = rec[0], A1 = rec[1], A2 = rec[2];
                Spp = fmaf(f, A0.y, A0.x);
                Spq = fmaf(f, A0.w, A0.z);
                Sqq = fmaf(f, A1.y, A1.x);
                e1 = fmaf(f, A1.w, A1.z);
                e2 = fmaf(f, A2.y, A2.x);
                r = fmaf(f, A2.w, A2.z);
                if (!TIME && g_v[5] == g_v[5]) {
                    // the lane's group-start interval is smooth: the arithmetic of a SPAN group
                    Spp = fmaf(xl, g_d[0], g_v[0]);
                    Spq = fmaf(xl, g_d[1], g_v[1]);
                    Sqq = fmaf(xl, g_d[2], g_v[2]);
                    e1 = fmaf(xl, g_d[3], g_v[3]);
                    e2 = fmaf(xl, g_d[4], g_v[4]);
                    r = fmaf(xl, g_d[5], g_v[5]);
                }
                if (__any(r != r)) {
                    asm volatile("; exact V'/V");
                    if (r != r) {
                        const float dT = (xh - c.xT_hi) + (xl - c.xT_lo);
                        r = __builtin_amdgcn_rcpf(fmaf(dT, c.kx, (dT >= 0.0f) ? s_plus : s_minus));
                    }
                }
            }
            const float z1 = z[2 * j], z2 = z[2 * j + 1];            // xi sqrt(dN)
            // noise plus bias through the shifted normals
            const float zb1 = (BIAS == kBiasConst) ? fmaf(adN, e1, z1) : z1;
            const float zb2 = (BIAS == kBiasConst) ? fmaf(adN, e2, z2) : z2;
            const float nphi = fmaf(Spp, zb1, Spq * zb2);
            const float npi = fmaf(Spq, zb1, Sqq * zb2);
            const float dx = fmaf(ps, c.dN, nphi);
            const float dpi = fmaf(fmaf(ps, ps, -6.0f), fmaf(ps, c.half_dN, r), npi);
            if (BIAS == kBiasConst) {
                const float dA = fmaf(a, fmaf(e1, z1, e2 * z2), half_a2_dN * fmaf(e1, e1, e2 * e2));
                zacc += (ALLPOS || Spp != 0.0f || Spq != 0.0f || Sqq != 0.0f) ? dA : 0.0f;
            }
            const float x0l = xl;
            xl += dx;
            pl += dpi;
            if (STEP_XS) xs = xh + xl;
            ps = ph + pl;
            // x <= 0: the sign of a rounded sum is that of the exact one, so this is xs <= 0
            const bool crossed = xl <= -xh;
            const bool ended = fabsf(ps) >= 0x1.6a09e8p+0f;
            const bool hit = live && (crossed || ended);
            if (hit) {
                float bh = xh, b0 = x0l, b1 = xl, bz = zacc;
                uint32_t nb = n + j;
                asm volatile("; passage event" : "+v"(bh), "+v"(b0), "+v"(b1), "+v"(nb), "+v"(bz));
                const double x0 = (double)bh + (double)b0;
                const double x1 = (double)bh + (double)b1;
                const double N_cross = (double)nb * dN + dN * (x0 / (x0 - x1));
                const double N_end = (double)(nb + 1) * dN;
                ev_code = (nb + 1) | (crossed ? 0u : kFlagEndedEarly);
                ev_N = crossed ? N_cross : N_end;
                ev_lnw = lnw - (double)bz;
            }
            live = live && !hit;
            fresh = fresh || hit;
        }
        n += G;
        lnw -= (double)zacc;
        if (fresh) retire(rt, rel, ev_code & ~kStepMask, ev_code & kStepMask, ev_N, ev_lnw);
        if (!STEP_XS) xs = xh + xl;
        xl = xl - (xs - xh);
        xh = xs;
        pl = pl - (ps - ph);
        ph = ps;
    };

    while (__any(has)) {
        const uint32_t left = wave_steps_left(has, n, I.max_steps);
        for (int k = 0; k < R.chunk; k += G) {
            if (!__any(live)) break;
            uint32_t w[2 * G];
#pragma unroll
            for (int q = 0; q < G / 2; ++q) philox_call((n >> 1) + (uint32_t)q, pre, R.key0, R.key1, w + 4 * q);
            float z[2 * G];
#pragma unroll
            for (int q = 0; q < 2 * G; q += 2) box_muller32(w[q], w[q + 1], c.m2ln2_dN, 0.0f, z[q], z[q + 1]);
            using T = std::integral_constant<bool, true>;
            using F = std::integral_constant<bool, false>;
            if constexpr (!TIME) {
                // the record of the lane's interval at the group start
                const float u0 = __builtin_amdgcn_fmed3f(fmaf(xh, c.inv_h, c.u_off), 0.0f, c.jtop);
                const int j0 = (int)u0;
                const float4 *rec = l_tab + 3 * j0;
                const float4 A0 = rec[0], A1 = rec[1], A2 = rec[2];
                const float fh = fmaf(xh, c.inv_h, c.u_off - (float)j0);   // the fraction at x = xh
                const float v0[6] = {A0.x, A0.z, A1.x, A1.z, A2.x, A2.z};
                const float d0[6] = {A0.y, A0.w, A1.y, A1.w, A2.y, A2.w};
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    g_v[q] = fmaf(fh, d0[q], v0[q]);
                    g_d[q] = d0[q] * c.inv_h;
                }
            }
            if ((uint32_t)k + G > left) {
                group(T(), F(), z);
            } else {
                if constexpr (!TIME) {
                    if (__builtin_amdgcn_ballot_w64(live && g_v[5] != g_v[5]) == 0) group(F(), T(), z);
                    else group(F(), F(), z);
                } else {
                    group(F(), F(), z);
                }
            }
        }
        if (!live) has = false;
        if (claim(!has, rel, cursor, n_traj, exhausted)) {
            has = true;
            live = true;
            xh = xs = x_in_hi;
            xl = x_in_lo;
            ph = ps = pi_in_hi;
            pl = pi_in_lo;
            lnw = 0.0;
            n = 0;
            pre = philox_pre(traj_offset + rel, I.instance, R.key0, R.key1);
        }
    }
}

// 2D staging: three double2 per node, then the Box-Muller tables.
__device__ __forceinline__ void stage_table64_2d(const Inst &I, double2 *l_tab)
{
    const int n = staged_nodes(I);
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) l_tab[i] = I.tab64_2d[I.n_tab > 1 ? i : i % 3];
    stage_bm(l_tab + 3 * n);
}

// FP32 2D staging: three float4 per node, the V'/V interval (last pair) scaled by dN/2 (NaN kept);
// a single node is staged twice with zero slopes and a NaN interval.
__device__ __forceinline__ void stage_table32_2d(const Inst &I, float4 *l_tab, float dN)
{
    const int n = staged_nodes(I);
    for (int i = threadIdx.x; i < 3 * n; i += blockDim.x) {
        float4 v = I.tab32_2d[I.n_tab > 1 ? i : i % 3];
        if (i % 3 == 2) {
            v.z *= 0.5f * dN;
            v.w *= 0.5f * dN;
        }
        l_tab[i] = v;
    }
}

// ---------------------------------------------------------------------------
// LDS layout of the kernels: [accumulators][noise table][control cells][node
// weights], each part starting on a 16-byte boundary.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ size_t align16(size_t b) { return (b + 15) & ~(size_t)15; }
// FP64: double2 per node; FP32: float4 per node plus the float2 V'/V interval
// LDS of a staged table: FP64 nodes (16 B) and the Box-Muller tables, or FP32 nodes and V'/V
// intervals (24 B per node).
__host__ __device__ __forceinline__ size_t tab_bytes(int precision, int n_tab)
{
    return align16((size_t)(n_tab > 1 ? n_tab : 2) * (precision == 0 ? 16 : 24)) + (precision == 0 ? kBmBytes : 0);
}
__host__ __device__ __forceinline__ size_t cell_bytes(int precision, int n_cells)
{
    return (size_t)n_cells * (precision == 0 ? 32 : 16);
}

template <int PREC>
__device__ __forceinline__ void stage_grid(const Inst &I, void *l_grid)
{
    const int nc = grid_cells(I);
    if (PREC == 0) {
        double2 *g = static_cast<double2 *>(l_grid);
        for (int i = threadIdx.x; i < 2 * nc; i += blockDim.x) g[i] = I.grid64[i];
    } else {
        float4 *g = static_cast<float4 *>(l_grid);
        for (int i = threadIdx.x; i < nc; i += blockDim.x) g[i] = I.grid32[i];
    }
}

// ---------------------------------------------------------------------------
// Single-problem kernels: a persistent grid over one instance.
// ---------------------------------------------------------------------------
__device__ __forceinline__ RetireTo retire_to(const EmParams &p, const LdsAcc &a)
{
    RetireTo r;
    r.d_N = p.d_N;
    r.d_lnw = p.d_lnw;
    r.d_steps = p.d_steps;
    r.cnt = a.cnt;
    r.sum = a.sum;
    r.nb = a.nb;
    r.hist = p.inst.hist;
    return r;
}

template <int PREC, int BIAS, int TAB, bool ALLPOS, int POT = kPotPiecewiseLinear>
__global__ void __launch_bounds__(1024) FPT_EM_OCCUPANCY em_kernel(EmParams p)
{
    static_assert(POT == kPotPiecewiseLinear || (PREC == 0 && (BIAS == kBiasNone || BIAS == kBiasConst)),
                  "the bump runs in FP64 only, without a learned bias");
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsAcc acc = lds_acc(smem, p.inst.hist.n_bins);
    unsigned char *l_tab = smem + align16(acc_bytes(p.inst.hist.n_bins));
    unsigned char *l_grid = l_tab + tab_bytes(PREC, p.inst.n_tab);
    zero_lds_acc(acc);
    if (PREC == 0) stage_table64(p.inst, reinterpret_cast<double2 *>(l_tab));
    else stage_table32(p.inst, reinterpret_cast<float4 *>(l_tab), (float)p.run.dN);
    if (BIAS == kBiasMlp) stage_grid<PREC>(p.inst, l_grid);
    if (BIAS == kBiasMlpExact && PREC == 0) stage_mlp64(p.inst.mlp_params, reinterpret_cast<double *>(l_grid));
    __syncthreads();
    const RetireTo rt = retire_to(p, acc);
    const ReplayTo rp{nullptr, nullptr, nullptr};
    if (PREC == 0)
        lanes_fp64<BIAS, TAB, ALLPOS, false, POT>(p.inst, p.run, reinterpret_cast<const double2 *>(l_tab),
                                                  reinterpret_cast<const double2 *>(l_grid), rt, rp, p.cursor,
                                                  p.n_traj, p.traj_offset);
    else
        lanes_fp32<BIAS, TAB, ALLPOS, false>(p.inst, p.run, reinterpret_cast<const float4 *>(l_tab),
                                             reinterpret_cast<const float4 *>(l_grid), rt, rp, p.cursor, p.n_traj,
                                             p.traj_offset);
    __syncthreads();
    flush_lds_acc(acc, p.inst.acc);
}

// 2D noise, FP64 or FP32 state: a persistent grid over one instance.
template <int PREC, int BIAS, bool ALLPOS, bool TIME>
__global__ void __launch_bounds__(1024) FPT_EM_OCCUPANCY em2d_kernel(EmParams p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const LdsAcc acc = lds_acc(smem, p.inst.hist.n_bins);
    unsigned char *l_tab = smem + align16(acc_bytes(p.inst.hist.n_bins));
    zero_lds_acc(acc);
    if (PREC == 0) stage_table64_2d(p.inst, reinterpret_cast<double2 *>(l_tab));
    else stage_table32_2d(p.inst, reinterpret_cast<float4 *>(l_tab), (float)p.run.dN);
    __syncthreads();
    const RetireTo rt = retire_to(p, acc);
    if (PREC == 0)
        lanes_fp64_2d<BIAS, ALLPOS, TIME>(p.inst, p.run, reinterpret_cast<const double2 *>(l_tab), rt, p.cursor,
                                          p.n_traj, p.traj_offset);
    else
        lanes_fp32_2d<BIAS, ALLPOS, TIME>(p.inst, p.run, reinterpret_cast<const float4 *>(l_tab), rt, p.cursor,
                                          p.n_traj, p.traj_offset);
    __syncthreads();
    flush_lds_acc(acc, p.inst.acc);
}

// Replay kernel: the listed trajectories with the tabulated control, scattering
// gradient factors onto the grid nodes (LDS, then global atomics).
template <int PREC, bool ALLPOS>
__global__ void __launch_bounds__(1024) FPT_EM_OCCUPANCY replay_kernel(ReplayParams p)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Inst &I = p.inst;
    unsigned char *l_tab = smem;
    unsigned char *l_grid = l_tab + tab_bytes(PREC, I.n_tab);
    double *l_G = reinterpret_cast<double *>(l_grid + cell_bytes(PREC, grid_cells(I)));
    const int n_nodes = I.g_n0 * I.g_n1;
    for (int i = threadIdx.x; i < n_nodes; i += blockDim.x) l_G[i] = 0.0;
    if (PREC == 0) stage_table64(I, reinterpret_cast<double2 *>(l_tab));
    else stage_table32(I, reinterpret_cast<float4 *>(l_tab), (float)p.run.dN);
    stage_grid<PREC>(I, l_grid);
    __syncthreads();
    RetireTo rt{};
    const ReplayTo rp{p.tail, l_G, p.mismatch};
    const uint64_t n_tail = *p.n_tail;
    if (PREC == 0)
        lanes_fp64<kBiasMlp, true, ALLPOS, true>(I, p.run, reinterpret_cast<const double2 *>(l_tab),
                                                 reinterpret_cast<const double2 *>(l_grid), rt, rp, p.cursor, n_tail,
                                                 0);
    else
        lanes_fp32<kBiasMlp, true, ALLPOS, true>(I, p.run, reinterpret_cast<const float4 *>(l_tab),
                                                 reinterpret_cast<const float4 *>(l_grid), rt, rp, p.cursor, n_tail,
                                                 0);
    __syncthreads();
    for (int i = threadIdx.x; i < n_nodes; i += blockDim.x)
        if (l_G[i] != 0.0) unsafeAtomicAdd(&p.d_G[i], l_G[i]);
}

// ---------------------------------------------------------------------------
// Batch kernel: a persistent grid over many instances.  Each instance has a
// trajectory cursor of its own (cursors[1 + i], over its whole range of the
// run).  The work list holds tickets, each sending a block to one instance
// (ordered so that the blocks spread over the instances in proportion to their
// estimated cost), then one entry per instance, longest estimated cost first.
// A block takes a ticket (cursors[0]) and skips it when its instance has no
// trajectory left; otherwise it stages that instance's table and histogram in
// LDS, and its waves claim the instance's trajectories from its global cursor
// until all are claimed, as in the single-instance kernel.  It then flushes the
// histogram and takes the next ticket; once the tickets are used up it joins
// any instance that still has trajectories left.  A block leaves an instance
// only when the instance has no trajectory left, so its lanes drain once per
// instance it works on, not once per ticket.  Every selection either finds an
// instance with trajectories left or ends the block's loop, and an instance
// found empty is never selected again: the loop ends.  The run parameters are
// read from device memory so that a captured graph can be replayed with a new
// seed or time step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool has_left(const WorkItem &W, unsigned long long *cursors)
{
    return __hip_atomic_load(&cursors[1 + W.inst], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < W.count;
}

template <int PREC, int BIAS, bool ALLPOS>
__global__ void __launch_bounds__(1024) FPT_EM_OCCUPANCY batch_kernel(const Inst *insts, const WorkItem *items,
                                                                      const BatchRun *brun,
                                                                      unsigned long long *cursors, int max_bins)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ long long s_sel;
    const RunArgs R = brun->run;
    const uint64_t n_items = brun->n_items, n_inst = brun->n_inst;
    uint64_t scan = 0;     // thread 0: the next per-instance entry to look at once the tickets are used up
    for (;;) {
        if (threadIdx.x == 0) {
            long long sel = -1;
            for (;;) {
                const uint64_t t = atomicAdd(&cursors[0], 1ull);
                if (t >= n_items) break;
                if (has_left(items[t], cursors)) {
                    sel = (long long)t;
                    break;
                }
            }
            for (; sel < 0 && scan < n_inst; ++scan)
                if (has_left(items[n_items + scan], cursors)) sel = (long long)(n_items + scan);
            s_sel = sel;
        }
        __syncthreads();
        const long long sel = s_sel;
        if (sel < 0) break;
        const WorkItem W = items[sel];
        const Inst I = insts[W.inst];
        const LdsAcc acc = lds_acc(smem, I.hist.n_bins);
        unsigned char *l_tab = smem + align16(acc_bytes(max_bins));
        zero_lds_acc(acc);
        if (PREC == 0) stage_table64(I, reinterpret_cast<double2 *>(l_tab));
        else stage_table32(I, reinterpret_cast<float4 *>(l_tab), (float)R.dN);
        __syncthreads();
        RetireTo rt;
        rt.d_N = nullptr;
        rt.d_lnw = nullptr;
        rt.d_steps = nullptr;
        rt.cnt = acc.cnt;
        rt.sum = acc.sum;
        rt.nb = acc.nb;
        rt.hist = I.hist;
        const ReplayTo rp{nullptr, nullptr, nullptr};
        if (PREC == 0)
            lanes_fp64<BIAS, true, ALLPOS, false>(I, R, reinterpret_cast<const double2 *>(l_tab), nullptr, rt, rp,
                                                  &cursors[1 + W.inst], W.count, W.begin);
        else
            lanes_fp32<BIAS, true, ALLPOS, false>(I, R, reinterpret_cast<const float4 *>(l_tab), nullptr, rt, rp,
                                                  &cursors[1 + W.inst], W.count, W.begin);
        __syncthreads();
        flush_lds_acc(acc, I.acc);
        __syncthreads();
    }
}

__global__ void zero_words_kernel(unsigned long long *ptr, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        ptr[i] = 0ull;
}

template <int PREC, int BIAS, int TAB, bool ALLPOS, int POT = kPotPiecewiseLinear>
const void *kptr() { return reinterpret_cast<const void *>(&em_kernel<PREC, BIAS, TAB, ALLPOS, POT>); }
template <int PREC, int BIAS, bool ALLPOS>
const void *bptr() { return reinterpret_cast<const void *>(&batch_kernel<PREC, BIAS, ALLPOS>); }

template <int PREC, int BIAS>
struct KTab {
    const void *p[3][2] = {{kptr<PREC, BIAS, 0, false>(), kptr<PREC, BIAS, 0, true>()},
                           {kptr<PREC, BIAS, 1, false>(), kptr<PREC, BIAS, 1, true>()},
                           {kptr<PREC, BIAS, 2, false>(), kptr<PREC, BIAS, 2, true>()}};
};

}  // namespace

size_t em_lds_bytes(int n_bins, int n_tab, int precision, int n_cells, bool mlp_exact)
{
    // the exact network stages its parameters (FP64 state) instead of the tabulated cells
    const size_t bias = mlp_exact ? (precision == 0 ? kMlpLdsBytes64 : 0) : cell_bytes(precision, n_cells);
    return align16(acc_bytes(n_bins)) + tab_bytes(precision, n_tab) + bias;
}

size_t replay_lds_bytes(int n_tab, int precision, int n_cells, int n_nodes)
{
    return tab_bytes(precision, n_tab) + cell_bytes(precision, n_cells) + (size_t)n_nodes * 8;
}

const void *em_kernel_ptr(int precision, int bias_kind, int tab_mode, bool all_pos, int pot_kind)
{
    const int tm = tab_mode < 0 ? 0 : tab_mode > 2 ? 2 : tab_mode;
    if (pot_kind == kPotGaussianBump) {
        // FP64, bias none or constant (fpt_create rejects the rest)
        constexpr int B = kPotGaussianBump;
        static const void *const tb[2][3][2] = {
            {{kptr<0, kBiasNone, 0, false, B>(), kptr<0, kBiasNone, 0, true, B>()},
             {kptr<0, kBiasNone, 1, false, B>(), kptr<0, kBiasNone, 1, true, B>()},
             {kptr<0, kBiasNone, 2, false, B>(), kptr<0, kBiasNone, 2, true, B>()}},
            {{kptr<0, kBiasConst, 0, false, B>(), kptr<0, kBiasConst, 0, true, B>()},
             {kptr<0, kBiasConst, 1, false, B>(), kptr<0, kBiasConst, 1, true, B>()},
             {kptr<0, kBiasConst, 2, false, B>(), kptr<0, kBiasConst, 2, true, B>()}}};
        return tb[bias_kind == kBiasConst ? 1 : 0][tm][all_pos ? 1 : 0];
    }
    static const KTab<0, kBiasNone> f0n;
    static const KTab<0, kBiasConst> f0c;
    static const KTab<0, kBiasMlp> f0m;
    static const KTab<0, kBiasMlpExact> f0x;
    static const KTab<1, kBiasNone> f1n;
    static const KTab<1, kBiasConst> f1c;
    static const KTab<1, kBiasMlp> f1m;
    static const KTab<1, kBiasMlpExact> f1x;
    const void *const(*t)[2];
    if (precision == 0)
        t = bias_kind == kBiasNone ? f0n.p : bias_kind == kBiasConst ? f0c.p : bias_kind == kBiasMlp ? f0m.p : f0x.p;
    else
        t = bias_kind == kBiasNone ? f1n.p : bias_kind == kBiasConst ? f1c.p : bias_kind == kBiasMlp ? f1m.p : f1x.p;
    return t[tm][all_pos ? 1 : 0];
}

hipError_t em_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream, bool mlp_exact)
{
    const size_t lds = em_lds_bytes(p.inst.hist.n_bins, p.inst.n_tab, precision, grid_cells(p.inst), mlp_exact);
    const void *fn = em_kernel_ptr(precision, mlp_exact ? kBiasMlpExact : p.inst.bias_kind, tab_mode(p.inst),
                                   p.inst.all_S_pos != 0, p.inst.pot_kind);
    EmParams pp = p;
    void *args[] = {&pp};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
}

size_t em2d_lds_bytes(int n_bins, int n_tab, int precision)
{
    // FP64: three double2 per node and the Box-Muller tables; FP32: three float4 per node
    return align16(acc_bytes(n_bins)) + (size_t)(n_tab > 1 ? n_tab : 2) * 48 + (precision == 0 ? kBmBytes : 0);
}

template <int PREC, int BIAS>
struct K2Tab {
    const void *p[2][2] = {{reinterpret_cast<const void *>(&em2d_kernel<PREC, BIAS, false, false>),
                            reinterpret_cast<const void *>(&em2d_kernel<PREC, BIAS, false, true>)},
                           {reinterpret_cast<const void *>(&em2d_kernel<PREC, BIAS, true, false>),
                            reinterpret_cast<const void *>(&em2d_kernel<PREC, BIAS, true, true>)}};
};

const void *em2d_kernel_ptr(int precision, int bias_kind, bool all_pos, bool time_axis)
{
    static const K2Tab<0, kBiasNone> d_n;
    static const K2Tab<0, kBiasConst> d_c;
    static const K2Tab<1, kBiasNone> f_n;
    static const K2Tab<1, kBiasConst> f_c;
    const bool c = bias_kind != kBiasNone;
    const void *const(*t)[2] = precision == 0 ? (c ? d_c.p : d_n.p) : (c ? f_c.p : f_n.p);
    return t[all_pos ? 1 : 0][time_axis ? 1 : 0];
}

hipError_t em2d_launch(const EmParams &p, int precision, int grid, int block, hipStream_t stream)
{
    const size_t lds = em2d_lds_bytes(p.inst.hist.n_bins, p.inst.n_tab, precision);
    const void *fn = em2d_kernel_ptr(precision, p.inst.bias_kind, p.inst.all_S_pos != 0, tab_mode(p.inst) == 2);
    EmParams pp = p;
    void *args[] = {&pp};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
}

const void *replay_kernel_ptr(int precision, bool all_pos)
{
    static const void *const t[2][2] = {
        {reinterpret_cast<const void *>(&replay_kernel<0, false>), reinterpret_cast<const void *>(&replay_kernel<0, true>)},
        {reinterpret_cast<const void *>(&replay_kernel<1, false>), reinterpret_cast<const void *>(&replay_kernel<1, true>)}};
    return t[precision ? 1 : 0][all_pos ? 1 : 0];
}

hipError_t replay_launch(const ReplayParams &p, int precision, int grid, int block, hipStream_t stream)
{
    const size_t lds = replay_lds_bytes(p.inst.n_tab, precision, grid_cells(p.inst), p.inst.g_n0 * p.inst.g_n1);
    const void *fn = replay_kernel_ptr(precision, p.inst.all_S_pos != 0);
    ReplayParams pp = p;
    void *args[] = {&pp};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
}

const void *batch_kernel_ptr(int precision, int bias_kind, bool all_pos)
{
    static const void *const t[2][2][2] = {
        {{bptr<0, kBiasNone, false>(), bptr<0, kBiasNone, true>()},
         {bptr<0, kBiasConst, false>(), bptr<0, kBiasConst, true>()}},
        {{bptr<1, kBiasNone, false>(), bptr<1, kBiasNone, true>()},
         {bptr<1, kBiasConst, false>(), bptr<1, kBiasConst, true>()}}};
    return t[precision ? 1 : 0][bias_kind == kBiasNone ? 0 : 1][all_pos ? 1 : 0];
}

hipError_t batch_launch(int precision, int bias_kind, bool all_pos, const Inst *insts, const WorkItem *items,
                        const BatchRun *run, unsigned long long *cursors, int max_bins, int max_tab, int grid,
                        int block, hipStream_t stream)
{
    const size_t lds = em_lds_bytes(max_bins, max_tab, precision, 0);
    const void *fn = batch_kernel_ptr(precision, bias_kind, all_pos);
    void *args[] = {&insts, &items, &run, &cursors, &max_bins};
    return hipLaunchKernel(fn, dim3(grid), dim3(block), args, lds, stream);
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
