// fpt_mlp.hip -- kernels of the learned importance-sampling control.
//
// The control amplitude a(phi, pi) is output 0 of a 2->64->64->2 network with
// tanh hidden layers and a linear output (FP32 parameters, evaluated in FP64),
// tabulated on a uniform grid of its normalised inputs and interpolated
// bilinearly by the Euler-Maruyama kernels.  Training minimises the second
// moment of the tail estimator, J(theta) = E[w_theta^2 1_T] (the log-weight
// variance on the tail under the lognormal weight model of Sec. 4.1), whose
// gradient at the sampling parameters is
//   dJ/dtheta = (1/n) sum_{paths in T} w^2 sum_k (-xi_k sqrt(dN)) da(x_k)/dtheta,
// with a(x) = sum_c beta_c(x) net(x_c) over the nodes c of x's cell.  The
// replay kernel (fpt_em.hip) accumulates the node weights
//   G_c = sum_T w^2 sum_k (-xi_k sqrt(dN)) beta_c(x_k);
// here the weights are propagated through the network at the nodes, and Adam
// (Kingma and Ba, 2015) updates the parameters.
//
// Parameter layout (row-major, out x in): W1[64x2] b1[64] W2[64x64] b2[64]
// W3[2x64] b3[2]; output 1 is unused with 1D noise (its gradient is 0).
#include "internal.hpp"

#include <hip/hip_runtime.h>
#include <math.h>

namespace fpt {
namespace {

constexpr int H = kMlpHidden;

__device__ __forceinline__ double grid_x(double lo, double hi, int n, int k)
{
    return lo + (hi - lo) * (double)k / (double)(n - 1);
}

// Hidden activations of the network at x (one wave of 64 lanes, lane = unit);
// returns output 0 in every lane.
__device__ __forceinline__ double net_forward(const float *p, double x0, double x1, double *l_h1, double *l_h2)
{
    const int t = threadIdx.x;
    double s = (double)p[kOffB1 + t];
    s += (double)p[2 * t] * x0;
    s += (double)p[2 * t + 1] * x1;
    l_h1[t] = tanh(s);
    __syncthreads();
    double s2 = (double)p[kOffB2 + t];
    for (int i = 0; i < H; ++i) s2 += (double)p[kOffW2 + t * H + i] * l_h1[i];
    l_h2[t] = tanh(s2);
    __syncthreads();
    double out = (double)p[kOffB3];
    for (int i = 0; i < H; ++i) out += (double)p[kOffW3 + i] * l_h2[i];
    return out;
}

// One block of 64 threads per grid node: the node value and its slots in the
// FP64 and FP32 cell tables (a node is a corner of up to four cells).
__global__ void __launch_bounds__(64) tabulate_kernel(const float *p, GridSpec g, double *node_a, double *grid64,
                                                      float *grid32)
{
    __shared__ double l_h1[H], l_h2[H];
    const int node = blockIdx.x;
    const int i = node / g.n1, j = node % g.n1;
    const double a = net_forward(p, grid_x(g.lo0, g.hi0, g.n0, i), grid_x(g.lo1, g.hi1, g.n1, j), l_h1, l_h2);
    if (threadIdx.x != 0) return;
    node_a[node] = a;
    const int n1c = g.n1 - 1;
    for (int ci = i - 1; ci <= i; ++ci) {
        if (ci < 0 || ci > g.n0 - 2) continue;
        for (int cj = j - 1; cj <= j; ++cj) {
            if (cj < 0 || cj > g.n1 - 2) continue;
            const int slot = 4 * (ci * n1c + cj) + 2 * (j - cj) + (i - ci);
            grid64[slot] = a;
            grid32[slot] = (float)a;
        }
    }
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Append the trajectories that crossed phi_end with deltaN >= tail_lo to the
// replay list with weight w^2, and add the weights to J_sum and the count to
// n_tail_total.
__global__ void tail_compact_kernel(const double *d_N, const double *d_lnw, const uint32_t *d_steps, uint64_t n,
                                    uint64_t traj_offset, double N_ref, double tail_lo, TailEntry *tail,
                                    unsigned long long *n_tail, unsigned long long *n_tail_total, double *J_sum)
{
    double j_local = 0.0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of iterations (the bound is rounded up to whole waves)
    const uint64_t n_up = (n + 63) & ~(uint64_t)63;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_up; i += stride) {
        bool in = false;
        double ww = 0.0;
        if (i < n) {
            in = (d_steps[i] & (kFlagCensored | kFlagEndedEarly)) == 0u && d_N[i] - N_ref >= tail_lo;
            if (in) ww = exp(2.0 * d_lnw[i]);
        }
        const uint64_t mask = __ballot(in);
        if (mask == 0) continue;
        const int leader = __ffsll((unsigned long long)mask) - 1;
        unsigned long long base = 0;
        if ((int)__lane_id() == leader) {
            base = atomicAdd(n_tail, (unsigned long long)__popcll(mask));
            atomicAdd(n_tail_total, (unsigned long long)__popcll(mask));
        }
        const uint32_t b_lo = (uint32_t)__shfl((int)(uint32_t)base, leader);
        const uint32_t b_hi = (uint32_t)__shfl((int)(uint32_t)(base >> 32), leader);
        if (in) {
            const uint64_t pos = (((uint64_t)b_hi << 32) | b_lo) + lanes_below(mask);
            tail[pos].traj = traj_offset + i;
            tail[pos].ww = ww;
            j_local += ww;
        }
    }
    for (int off = 32; off > 0; off >>= 1) j_local += __shfl_down(j_local, off);
    if (__lane_id() == 0 && j_local != 0.0) unsafeAtomicAdd(J_sum, j_local);
}

// Backward pass at every node: work = [H1 | H2 | D2 | G1], each n_nodes x 64,
// with D2 = G_c W3 (1 - h2^2) and G1 = (W2^T D2)(1 - h1^2).
__device__ __forceinline__ double inv_den(double n_scale, const double *d_den)
{
    const double den = d_den ? *d_den : n_scale;
    return den != 0.0 ? 1.0 / den : 0.0;
}

__global__ void __launch_bounds__(64) backprop_node_kernel(const float *p, GridSpec g, const double *G,
                                                           double n_scale, const double *d_den, double *work)
{
    __shared__ double l_h1[H], l_h2[H], l_d2[H];
    const int node = blockIdx.x, t = threadIdx.x;
    const int n_nodes = g.n0 * g.n1;
    const int i = node / g.n1, j = node % g.n1;
    (void)net_forward(p, grid_x(g.lo0, g.hi0, g.n0, i), grid_x(g.lo1, g.hi1, g.n1, j), l_h1, l_h2);
    const double Gc = G[node] * inv_den(n_scale, d_den);
    const double h1 = l_h1[t], h2 = l_h2[t];
    const double d2 = Gc * (double)p[kOffW3 + t] * (1.0 - h2 * h2);
    l_d2[t] = d2;
    __syncthreads();
    double d1 = 0.0;
    for (int k = 0; k < H; ++k) d1 += l_d2[k] * (double)p[kOffW2 + k * H + t];
    double *H1 = work, *H2 = work + (size_t)n_nodes * H, *D2 = work + 2 * (size_t)n_nodes * H,
           *G1 = work + 3 * (size_t)n_nodes * H;
    H1[(size_t)node * H + t] = h1;
    H2[(size_t)node * H + t] = h2;
    D2[(size_t)node * H + t] = d2;
    G1[(size_t)node * H + t] = d1 * (1.0 - h1 * h1);
}

// One thread per parameter: the sum over nodes (fixed order) of its factors.
__global__ void backprop_param_kernel(GridSpec g, const double *G, double n_scale, const double *d_den,
                                      const double *work, float *grad)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= kMlpParams) return;
    const double inv = inv_den(n_scale, d_den);
    const int n_nodes = g.n0 * g.n1;
    const double *H1 = work, *H2 = work + (size_t)n_nodes * H, *D2 = work + 2 * (size_t)n_nodes * H,
                 *G1 = work + 3 * (size_t)n_nodes * H;
    double s = 0.0;
    if (q < kOffB1) {                         // W1[u, k]
        const int u = q / 2, k = q % 2;
        for (int c = 0; c < n_nodes; ++c) {
            const double x = k == 0 ? grid_x(g.lo0, g.hi0, g.n0, c / g.n1) : grid_x(g.lo1, g.hi1, g.n1, c % g.n1);
            s += G1[(size_t)c * H + u] * x;
        }
    } else if (q < kOffW2) {                  // b1[u]
        const int u = q - kOffB1;
        for (int c = 0; c < n_nodes; ++c) s += G1[(size_t)c * H + u];
    } else if (q < kOffB2) {                  // W2[u, v]
        const int u = (q - kOffW2) / H, v = (q - kOffW2) % H;
        for (int c = 0; c < n_nodes; ++c) s += D2[(size_t)c * H + u] * H1[(size_t)c * H + v];
    } else if (q < kOffW3) {                  // b2[u]
        const int u = q - kOffB2;
        for (int c = 0; c < n_nodes; ++c) s += D2[(size_t)c * H + u];
    } else if (q < kOffW3 + H) {              // W3[0, v]
        const int v = q - kOffW3;
        for (int c = 0; c < n_nodes; ++c) s += G[c] * inv * H2[(size_t)c * H + v];
    } else if (q == kOffB3) {                 // b3[0]
        for (int c = 0; c < n_nodes; ++c) s += G[c] * inv;
    }                                         // W3[1, .] and b3[1] feed the unused output
    grad[q] = (float)s;
}

__global__ void scale_copy_kernel(const double *src, double scale, double *dst, size_t n)
{
    const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i] * scale;
}

__global__ void adam_kernel(float *theta, float *m, float *v, const float *grad, int n, double lr, double b1,
                            double b2, double eps, double bc1, double bc2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double g = (double)grad[q];
    const double mq = b1 * (double)m[q] + (1.0 - b1) * g;
    const double vq = b2 * (double)v[q] + (1.0 - b2) * g * g;
    m[q] = (float)mq;
    v[q] = (float)vq;
    const double step = lr * (mq / bc1) / (sqrt(vq / bc2) + eps);
    theta[q] = (float)((double)theta[q] - step);
}

}  // namespace

hipError_t mlp_tabulate(const float *params, const GridSpec &g, double *node_a, double2 *grid64, float4 *grid32,
                        hipStream_t stream)
{
    hipLaunchKernelGGL(tabulate_kernel, dim3(g.n0 * g.n1), dim3(H), 0, stream, params, g, node_a,
                       reinterpret_cast<double *>(grid64), reinterpret_cast<float *>(grid32));
    return hipGetLastError();
}

hipError_t mlp_tail_compact(const double *d_N, const double *d_lnw, const uint32_t *d_steps, uint64_t n,
                            uint64_t traj_offset, double N_ref, double tail_lo, TailEntry *tail,
                            unsigned long long *n_tail, unsigned long long *n_tail_total, double *J_sum,
                            hipStream_t stream)
{
    const int block = 256;
    uint64_t blocks = (n + block - 1) / block;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(tail_compact_kernel, dim3((unsigned)blocks), dim3(block), 0, stream, d_N, d_lnw, d_steps, n,
                       traj_offset, N_ref, tail_lo, tail, n_tail, n_tail_total, J_sum);
    return hipGetLastError();
}

hipError_t mlp_backprop(const float *params, const GridSpec &g, const double *G, double n_scale,
                        const double *d_den, double *work, float *grad, hipStream_t stream)
{
    hipLaunchKernelGGL(backprop_node_kernel, dim3(g.n0 * g.n1), dim3(H), 0, stream, params, g, G, n_scale, d_den,
                       work);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(backprop_param_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, stream, g, G, n_scale,
                       d_den, work, grad);
    return hipGetLastError();
}

hipError_t mlp_scale_copy(const double *src, double scale, double *dst, size_t n, hipStream_t stream)
{
    hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src, scale, dst, n);
    return hipGetLastError();
}

hipError_t mlp_adam(float *params, float *m, float *v, const float *grad, int n, double lr, double beta1,
                    double beta2, double eps, double bc1, double bc2, hipStream_t stream)
{
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, params, m, v, grad, n, lr, beta1,
                       beta2, eps, bc1, bc2);
    return hipGetLastError();
}

}  // namespace fpt
