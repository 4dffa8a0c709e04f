// Coarse-space deflation of the FP32 inner solves (not in the paper).
//
// The slowly converging part of GMRES on the multiple-scattering system is
// the long-range coupling of the patches' total charges, whose smooth global
// modes the coarse (monopole) model of coarse.hip describes. With Z the
// N x k orthonormal basis of the polynomials of degree <= 3 in the patch
// centres (k = 16 on the sphere), placed in every patch's e_0 coefficient,
// and T = Z^T C Z the coarse operator C = I + chi0 G restricted to it, the
// right preconditioner
//
//     M^{-1} v = v + Z (T^{-1} - I) Z^T v
//
// (a spectral deflation preconditioner in the sense of Erhel, Burrage and
// Pohl, with T from the coarse model instead of the system itself) moves the
// modes Z spans towards 1. T costs one all-pairs pass over the centres that
// carries all k columns at once; applying M^{-1} costs k dot products and one
// update of the e_0 coefficients.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace nce {

constexpr int kDefl = 16;  // basis columns (padded with zeros when the layout gives fewer); equals
                           // the count of deflate_basis.cpp

struct Deflation {
    int N = 0, K = 0, k = 0;         // k = independent basis columns (<= kDefl)
    double* Z = nullptr;             // N x kDefl, row-major (device)
    double* Minv = nullptr;          // kDefl x kDefl: T^{-1} - I on the first k rows/columns (device)
    double* partial = nullptr;       // reduction partials (device)
    std::vector<double> T;           // k x k coarse operator on the basis (host, row-major)

    Deflation() = default;
    Deflation(const Deflation&) = delete;
    Deflation& operator=(const Deflation&) = delete;
    ~Deflation();
    // Builds Z from the centres (frames: N x 9 host, (c, e1, e2) per patch) and
    // T from the coarse model (chi0, problem); frames_dev is the device copy.
    void build(hipStream_t s, int N, int K, int problem, double chi0, const std::vector<double>& frames,
               const double* frames_dev);
    // out = M^{-1} in for N x K vectors (out may equal in).
    hipError_t apply(hipStream_t s, const double* in, double* out) const;
};

// Host: orthonormal basis (modified Gram-Schmidt, twice) of the monomials of
// degree <= 3 in the centres c_i = frames[9 i .. 9 i + 2]; returns the number
// of independent columns and fills Z (N x kDefl, zero beyond them).
int deflation_basis(const std::vector<double>& frames, int N, std::vector<double>& Z);
// Host: G = Z^T S on the first k columns (Z, S: N x kDefl); k x k row-major.
void deflation_gram(const std::vector<double>& Z, const std::vector<double>& S, int N, int k,
                    std::vector<double>& G);

// S_i = sum_{j != i} G(c_i, c_j) Z_j for the kDefl columns at once (FP32 pair
// sums, FP64 accumulation); Z, S: N x kDefl row-major device arrays.
void coarse_multi(hipStream_t s, int problem, int N, const double* frames_dev, const double* Z, double* S);

}  // namespace nce
