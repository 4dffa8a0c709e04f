// Monopole (coarse) model of the system: one unknown a_i per patch,
//     a_i + chi0 sum_{j != i} G(c_i, c_j) a_j = 1,
// solved on the device; see coarse.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace nce {

struct CoarseSolver {
    int N, problem;
    double chi0;
    int maxit;
    int nsplit = 1, chunk = 0;
    float4* src = nullptr;
    double* part = nullptr;
    double* V = nullptr;
    double* h = nullptr;
    double* rpart = nullptr;
    double* scal = nullptr;

    CoarseSolver(int N, int problem, double chi0, int maxit);
    ~CoarseSolver();
    CoarseSolver(const CoarseSolver&) = delete;
    CoarseSolver& operator=(const CoarseSolver&) = delete;
    // y = C a (device vectors of N doubles); frames: N x 9 device (c, e1, e2)
    void apply(hipStream_t s, const double* frames, const double* a, double* y);
    // a = C^{-1} 1 to relative residual tol (GMRES); returns the iterations used
    int solve(hipStream_t s, const double* frames, double tol, double* a);
};

}  // namespace nce
