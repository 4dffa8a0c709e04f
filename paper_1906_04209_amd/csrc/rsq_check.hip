// Accuracy of the gfx950 FP64 reciprocal square root estimate
// (v_rsq_f64) and of one first-order and one second-order correction, over
// 2^20 arguments log-uniform in [1e-9, 3] (the squared half-distances of the
// pair kernels), against a long-double host reference. Built on request with
// the issue-cost probe (python -m paper_1906_04209_amd.build --rates); not
// part of the library.
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
__global__ void k(const double* x, double* y0, double* y1, double* y2, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    const double y = __builtin_amdgcn_rsq(v);
    const double e = fma(-v * y, y, 1.0);
    y0[i] = y;
    y1[i] = fma(y * 0.5, e, y);
    y2[i] = fma(y * e, fma(e, 0.375, 0.5), y);
}
int main() {
    const int n = 1 << 20;
    std::vector<double> x(n), a(n), b(n), c(n);
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u(-9.0, 0.5);
    for (int i = 0; i < n; ++i) x[i] = std::pow(10.0, u(g));
    double *dx, *d0, *d1, *d2;
    if (hipMalloc(&dx, n * 8) || hipMalloc(&d0, n * 8) || hipMalloc(&d1, n * 8) || hipMalloc(&d2, n * 8)) return 1;
    hipMemcpy(dx, x.data(), n * 8, hipMemcpyHostToDevice);
    hipLaunchKernelGGL(k, dim3(n / 256), dim3(256), 0, 0, dx, d0, d1, d2, n);
    if (hipDeviceSynchronize() != hipSuccess) return 2;
    hipMemcpy(a.data(), d0, n * 8, hipMemcpyDeviceToHost);
    hipMemcpy(b.data(), d1, n * 8, hipMemcpyDeviceToHost);
    hipMemcpy(c.data(), d2, n * 8, hipMemcpyDeviceToHost);
    long double m0 = 0, m1 = 0, m2 = 0, s1 = 0;
    for (int i = 0; i < n; ++i) {
        const long double r = 1.0L / std::sqrt((long double)x[i]);
        m0 = std::max(m0, std::fabs(a[i] / r - 1));
        const long double e1 = b[i] / r - 1;
        m1 = std::max(m1, std::fabs(e1));
        s1 += e1;
        m2 = std::max(m2, std::fabs(c[i] / r - 1));
    }
    printf("rsq_f64 estimate max rel err %.3Le (2^%.1Lf)\n", m0, std::log2(m0));
    printf("first-order corrected max rel err %.3Le (2^%.1Lf), mean %.3Le\n", m1, std::log2(m1), s1 / n);
    printf("second-order corrected max rel err %.3Le (2^%.1Lf)\n", m2, std::log2(m2));
    return 0;
}
