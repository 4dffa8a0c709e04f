// Issue cost of single VALU instructions on the GPU, in lane-cycles at the
// nominal clock (256 CUs x 64 lanes x 2.4 GHz): a grid of 4096 blocks x 256
// threads runs 8 independent dependency chains of one instruction per thread;
// cost = nominal lane-cycles per second / measured lane-ops per second. These
// costs price the instruction mix of the Green's-function inner loops.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>

#define CHK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s line %d\n", hipGetErrorString(e), __LINE__); exit(1);} } while (0)

constexpr int ITERS = 2048;
constexpr int CH = 8;

template <int OP>
__global__ __launch_bounds__(256) void k(float* out32, double* out64, float seed) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    float x[CH];
    double d[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) { x[c] = seed + 0.01f * c + 1e-7f * tid; d[c] = (double)x[c]; }
    for (int it = 0; it < ITERS; ++it) {
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            if (OP == 0) x[c] = __builtin_fmaf(x[c], 0.999f, 0.001f);
            if (OP == 1) x[c] = __builtin_amdgcn_rsqf(x[c]);
            if (OP == 2) x[c] = __builtin_amdgcn_logf(x[c]);
            if (OP == 3) x[c] = __builtin_amdgcn_rcpf(x[c]);
            if (OP == 4) d[c] = __builtin_fma(d[c], 0.999, 0.001);
            if (OP == 5) d[c] = __builtin_amdgcn_rcp(d[c]);
            if (OP == 6) d[c] = __builtin_amdgcn_rsq(d[c]);
            if (OP == 7) d[c] = __builtin_amdgcn_frexp_mant(d[c]);
            if (OP == 8) x[c] = __builtin_amdgcn_sqrtf(x[c]);
            if (OP == 9) x[c] = __builtin_amdgcn_exp2f(x[c]);
            if (OP == 10) x[c] = __builtin_bit_cast(float, (__builtin_bit_cast(unsigned, x[c]) ^ 0x5bd1e995u) + 0x9e3779b9u);
            if (OP == 11) d[c] = d[c] * 0.999 + 0.5;  // fma-contracted; see 12
            if (OP == 12) d[c] = d[c] + 0.001;
            if (OP == 13) x[c] = (float)(d[c] = (double)x[c] + 1e-3);
            if (OP == 14) x[c] = x[c] > 1.0f ? x[c] - 0.5f : x[c] + 0.25f;
            if (OP == 15) x[c] = x[c] * 0.999f;
        }
    }
    float s = 0.f;
    double t = 0.0;
#pragma unroll
    for (int c = 0; c < CH; ++c) { s += x[c]; t += d[c]; }
    out32[tid] = s;
    out64[tid] = t;
}

template <int OP>
void run(const char* name, float* o32, double* o64, int blocks) {
    hipEvent_t a, b;
    CHK(hipEventCreate(&a)); CHK(hipEventCreate(&b));
    hipLaunchKernelGGL(k<OP>, dim3(blocks), dim3(256), 0, 0, o32, o64, 1.5f);
    CHK(hipGetLastError());
    CHK(hipEventRecord(a));
    const int reps = 5;
    for (int r = 0; r < reps; ++r) hipLaunchKernelGGL(k<OP>, dim3(blocks), dim3(256), 0, 0, o32, o64, 1.5f);
    CHK(hipEventRecord(b));
    CHK(hipEventSynchronize(b));
    float ms; CHK(hipEventElapsedTime(&ms, a, b));
    const double lane_ops = (double)reps * blocks * 256 * ITERS * CH;
    const double rate = lane_ops / (ms * 1e-3);
    const double lane_cycles = 256.0 * 64 * 2.4e9;
    printf("%-18s %8.3f ms  %.3e lane-ops/s  cost %.2f lane-cycles per op (at 2.4 GHz, 256 CUs)\n", name, ms / reps, rate,
           lane_cycles / rate);
    fflush(stdout);
}

int main() {
    const int blocks = 256 * 16;
    float* o32; double* o64;
    CHK(hipMalloc(&o32, sizeof(float) * blocks * 256));
    CHK(hipMalloc(&o64, sizeof(double) * blocks * 256));
    hipDeviceProp_t p; CHK(hipGetDeviceProperties(&p, 0));
    printf("device %s CUs %d clock %d kHz\n", p.gcnArchName, p.multiProcessorCount, p.clockRate);
    run<0>("v_fma_f32", o32, o64, blocks);
    run<1>("v_rsq_f32", o32, o64, blocks);
    run<2>("v_log_f32", o32, o64, blocks);
    run<3>("v_rcp_f32", o32, o64, blocks);
    run<8>("v_sqrt_f32", o32, o64, blocks);
    run<9>("v_exp_f32", o32, o64, blocks);
    run<4>("v_fma_f64", o32, o64, blocks);
    run<5>("v_rcp_f64", o32, o64, blocks);
    run<6>("v_rsq_f64", o32, o64, blocks);
    run<7>("v_frexp_mant_f64", o32, o64, blocks);
    run<10>("v_xor+v_add_u32 (2)", o32, o64, blocks);
    run<12>("v_add_f64", o32, o64, blocks);
    run<13>("cvt f32->f64->f32+add", o32, o64, blocks);
    run<14>("cmp+cndmask+add", o32, o64, blocks);
    run<15>("v_mul_f32", o32, o64, blocks);
    CHK(hipFree(o32)); CHK(hipFree(o64));
    return 0;
}
