// valu_rates.hip -- measurement helper (not part of the library): the issue rate of single
// instruction kinds on one GPU, as wave-instructions per cycle per SIMD at a nominal 2.4 GHz.
// Each thread runs 8 independent chains of one kind, registers only; the one store per thread
// is in bounds (grid x block floats).  Build and run:
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       tests/helpers/valu_rates.hip -o /tmp/valu_rates && /tmp/valu_rates
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>

#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); return 1; } } while (0)

template <int OP>
__global__ void __launch_bounds__(256) probe(float *out, int iters)
{
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    float f[8];
    double d[8];
    const float ra = 0.9999f + 1e-9f * (float)threadIdx.x, rb = 1e-4f * (float)(threadIdx.x & 3);
    uint32_t u[8];
    for (int k = 0; k < 8; ++k) {
        f[k] = 1.0f + 1e-3f * (float)(threadIdx.x + k);
        d[k] = 1.0 + 1e-3 * (double)(threadIdx.x + k);
        u[k] = 0x9E3779B9u * (uint32_t)(gid + k + 1);
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            if (OP == 0) f[k] = fmaf(f[k], 0.9999f, 1e-4f);                       // v_fma_f32
            if (OP == 1) d[k] = fma(d[k], 0.9999, 1e-4);                          // v_fma_f64
            if (OP == 2) { uint64_t p = (uint64_t)u[k] * 0xD2511F53u; u[k] = (uint32_t)(p >> 32) ^ (uint32_t)p; }  // v_mad_u64_u32 + xor
            if (OP == 3) f[k] = __builtin_amdgcn_logf(f[k] + 2.0f);               // v_log_f32 + add
            if (OP == 4) f[k] = __builtin_amdgcn_sinf(f[k]);                      // v_sin_f32
            if (OP == 5) f[k] = f[k] * 0.9999f + f[(k + 1) & 7] * 1e-6f;          // mul + fma mix
            if (OP == 6) u[k] = u[k] ^ (u[k] >> 3) ^ 0x5bd1e995u;                  // int ALU (bitop3/shift)
            if (OP == 7) f[k] = fmaf(f[k], ra, rb);                               // fma, register operands
            if (OP == 8) { f[k] = fmaf(f[k], ra, rb); d[k] = fma(d[k], 1.0000001, 1e-9); }  // f32 + f64 interleaved
        }
    }
    float s = 0.0f;
    for (int k = 0; k < 8; ++k) s += f[k] + (float)d[k] + (float)(u[k] & 0xff);
    out[gid] = s;
}

template <int OP>
int run(const char *name, float *d_out, int grid, int block, int iters, int instr_per_item)
{
    hipEvent_t a, b;
    CHK(hipEventCreate(&a));
    CHK(hipEventCreate(&b));
    hipLaunchKernelGGL(probe<OP>, dim3(grid), dim3(block), 0, 0, d_out, 16);
    CHK(hipGetLastError());
    CHK(hipDeviceSynchronize());
    CHK(hipEventRecord(a));
    hipLaunchKernelGGL(probe<OP>, dim3(grid), dim3(block), 0, 0, d_out, iters);
    CHK(hipEventRecord(b));
    CHK(hipEventSynchronize(b));
    float ms = 0;
    CHK(hipEventElapsedTime(&ms, a, b));
    const double waves = (double)grid * block / 64.0;
    const double winstr = waves * iters * 8.0 * instr_per_item;   // wave-instructions of the probed kind
    const double cycles = ms * 1e-3 * 2.4e9;
    printf("%-22s %8.2f ms  wave-instr per cycle per SIMD: %.3f\n", name, ms, winstr / cycles / 1024.0);
    fflush(stdout);
    return 0;
}

int main()
{
    int dev = 0;
    CHK(hipSetDevice(dev));
    int cus = 0;
    CHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int block = 256, grid = cus * 16;       // 64 waves per CU: 16 per SIMD
    float *d_out = nullptr;
    CHK(hipMalloc(&d_out, sizeof(float) * grid * block));
    const int it = 20000;
    if (run<0>("fma_f32", d_out, grid, block, it, 1)) return 1;
    if (run<1>("fma_f64", d_out, grid, block, it / 2, 1)) return 1;
    if (run<2>("mad_u64_u32(+xor)", d_out, grid, block, it / 4, 1)) return 1;
    if (run<3>("log_f32(+add)", d_out, grid, block, it / 4, 1)) return 1;
    if (run<4>("sin_f32", d_out, grid, block, it / 4, 1)) return 1;
    if (run<5>("mul+fma f32", d_out, grid, block, it, 2)) return 1;
    if (run<6>("int xor/shift", d_out, grid, block, it, 1)) return 1;
    if (run<7>("fma_f32 (vgpr operands)", d_out, grid, block, it, 1)) return 1;
    if (run<7>("fma_f32 (vgpr, 8 w/SIMD)", d_out, cus * 8, block, it, 1)) return 1;
    if (run<7>("fma_f32 (vgpr, 4 w/SIMD)", d_out, cus * 4, block, it, 1)) return 1;
    if (run<8>("fma f32+f64 pairs", d_out, grid, block, it / 2, 2)) return 1;
    CHK(hipFree(d_out));
    return 0;
}
