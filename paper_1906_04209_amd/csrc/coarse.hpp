// Monopole (coarse) model of the system: one unknown a_i per patch,
//     a_i + sum_{j != i} G(c_i, c_j) chi0_j a_j = 1
// (chi0_j = chi0 for one patch radius), solved on the device; see coarse.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <vector>

#include "deflate.hpp"

namespace nce {

struct CoarseSolver {
    int N, problem;          // N: the largest layout the solver takes
    double chi0;
    int maxit;
    float4* src = nullptr;
    double* part = nullptr;
    double* V = nullptr;
    double* h = nullptr;
    double* rpart = nullptr;
    double* scal = nullptr;
    double* tmp = nullptr;   // N doubles: the preconditioned Krylov vector
    double* chi = nullptr;   // per-patch charges chi0_j (N doubles) after set_charges; else chi0 for all
    // y = C a for the solver's own layout (n = N) by a faster route when set:
    // the far field through the configuration's tree instead of all pairs
    std::function<void(hipStream_t, const double*, double*)> fast_apply;

    CoarseSolver(int N, int problem, double chi0, int maxit);
    ~CoarseSolver();
    CoarseSolver(const CoarseSolver&) = delete;
    CoarseSolver& operator=(const CoarseSolver&) = delete;
    // Per-patch charges chi0_j (a layout of several patch radii: each patch's
    // radius's chi0), n <= N values in the layout's patch order; replaces the
    // common chi0 in later applies and solves.
    void set_charges(hipStream_t s, const std::vector<double>& chi0_patch);
    // y = C a for a layout of n <= N centres (device vectors of n doubles);
    // frames: n x 9 device (c, e1, e2)
    void apply(hipStream_t s, int n, const double* frames, const double* a, double* y);
    // The pieces of a tree apply of C: q = chi0_j a_j in FP32 (the sources'
    // charges, n values), then y = a + u from the summed field u (n floats).
    hipError_t charges32(hipStream_t s, int n, const double* a, float* q) const;
    static hipError_t finish32(hipStream_t s, int n, const double* a, const float* u, double* y);
    // a = C^{-1} 1 to relative residual tol (GMRES); returns the iterations
    // used. With defl (built for this layout, n patches) GMRES runs on
    // C M^{-1} with the deflation's M^{-1} acting on the amplitudes.
    int solve(hipStream_t s, int n, const double* frames, double tol, double* a, const Deflation* defl = nullptr);
};

}  // namespace nce
