// Per-eps precompute steps on the GPU (see precompute_gpu.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <vector>

#include "precompute.hpp"

namespace nce {

// The patch's fine grid on the device: points (nf x 3) and W B (nf x K,
// quadrature weight times basis density).
struct GpuFine {
    hipStream_t stream;
    int nf, K;
    double* fxyz = nullptr;
    double* wB = nullptr;
    GpuFine(hipStream_t s, const std::vector<double>& fxyz, const std::vector<double>& wB, int K);
    ~GpuFine();
    GpuFine(const GpuFine&) = delete;
    GpuFine& operator=(const GpuFine&) = delete;
};

struct IdResult {
    int p = 0;              // rank
    int ell = 0;            // sketch rows used
    std::vector<int> piv;   // column order; the first p are the skeleton
    std::vector<double> T;  // p x K
};

// Randomized ID of G(x^t, x^f) (training points txyz, nt x 3, on the sphere)
// and T = Pi W B, all on the device; rank by tol_id relative to the largest
// pivot; sketch rows start at ell0 and double while p >= ell - 48.
IdResult interpolative_decomposition_gpu(const GpuFine& fine, int problem, const std::vector<double>& txyz,
                                         double tol_id, int ell0, uint64_t seed);

// {max |full - skeleton|, max |full|} of the outgoing field at held-out points
// hxyz: full fine-grid quadrature against the skeleton (skel_xyz, p x 3) with T.
std::vector<double> field_check_gpu(const GpuFine& fine, int problem, const std::vector<double>& hxyz,
                                    const std::vector<double>& skel_xyz, const std::vector<double>& T);

// nmodes dense systems A_m X = F_m (n x n row-major, n x nrhs_max row-major,
// nrhs[m] columns used), solved by LU with partial pivoting, one block per
// system; F is overwritten by the solutions.
void modal_solve_gpu(hipStream_t s, int n, int nmodes, std::vector<double>& A, std::vector<double>& F,
                     const std::vector<int>& nrhs, int nrhs_max);

// The device steps of build_tables (modal solves, IDs, checks) on stream s.
std::unique_ptr<PrecomputeDevice> make_gpu_precompute(hipStream_t s);

}  // namespace nce
