// Coarse-space deflation of the FP32 inner solves (not in the paper).
//
// The slowly converging part of GMRES on the multiple-scattering system is
// the long-range coupling of the patches' total charges, whose smooth global
// modes the coarse (monopole) model of coarse.hip describes. With Z the
// N x k orthonormal basis of the polynomials of degree <= 3 in the patch
// centres (k = 16 on the sphere), placed in every patch's e_0 coefficient,
// and T = Z^T C Z the coarse operator C = I + chi0 G restricted to it (I + G D,
// D = diag(chi0_j), for patches of several radii), the
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
constexpr int kDeflMinN = 64;  // configurations with fewer patches are not deflated

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
    // T from the coarse model (chi0, problem; chi_patch, when given, N
    // per-patch charges in place of chi0, for patches of several radii);
    // frames_dev is the device copy.
    void build(hipStream_t s, int N, int K, int problem, double chi0, const std::vector<double>& frames,
               const double* frames_dev, const std::vector<double>* chi_patch = nullptr);
    // out = M^{-1} in for N x K vectors (out may equal in).
    hipError_t apply(hipStream_t s, const double* in, double* out) const { return apply_stride(s, in, out, K); }
    // the same for N x stride vectors (stride 1: one value per patch, as the
    // coarse model's amplitudes)
    hipError_t apply_stride(hipStream_t s, const double* in, double* out, int stride) const;
};

// One configuration's deflation data on the host: Z (N x kDefl, zero beyond
// the k independent columns) and M = T^{-1} - I (kDefl x kDefl, zero beyond
// k); T (k x k) into *T when given. With chi_patch (N per-patch charges) the
// coarse operator is I + G D, D = diag(chi_patch), instead of I + chi0 G.
// Returns k; N < kDeflMinN (zero Z and M) or a singular T (zero M) give 0,
// and the apply is then the identity.
int deflation_member(hipStream_t s, int N, int problem, double chi0, const std::vector<double>& frames,
                     const double* frames_dev, std::vector<double>& Z, std::vector<double>& M,
                     std::vector<double>* T, const std::vector<double>* chi_patch = nullptr);

// M^{-1} for ncfg configurations stored one after another (configuration c =
// patches [pseg[c], pseg[c + 1]), patch_cfg[i] = c; Z: npatch x kDefl, M: ncfg
// x kDefl x kDefl, d: ncfg x kDefl scratch; all device), in place on v (npatch
// x K, e_0 coefficients changed). Configurations with active[c] = 0 (active
// may be null) are left unchanged. Two launches, no allocation.
hipError_t deflation_apply_batched(hipStream_t s, int ncfg, int64_t npatch, int K, const int64_t* pseg,
                                   const int* patch_cfg, const double* Z, const double* M, const int* active,
                                   double* d, double* v);

// Host: orthonormal basis (modified Gram-Schmidt, twice) of the monomials of
// degree <= 3 in the centres c_i = frames[9 i .. 9 i + 2]; returns the number
// of independent columns and fills Z (N x kDefl, zero beyond them).
int deflation_basis(const std::vector<double>& frames, int N, std::vector<double>& Z);
// Host: G = Z^T S on the first k columns (Z, S: N x kDefl); k x k row-major.
void deflation_gram(const std::vector<double>& Z, const std::vector<double>& S, int N, int k,
                    std::vector<double>& G);

// S_i = sum_{j != i} G(c_i, c_j) Z_j for the kDefl columns at once (FP32 pair
// sums, FP64 accumulation); Z, S: N x kDefl row-major device arrays.
// Synchronous, with its own scratch.
void coarse_multi(hipStream_t s, int problem, int N, const double* frames_dev, const double* Z, double* S);

// Device scratch of coarse_multi_enqueue, reusable across configurations in
// stream order; reserve(N) before enqueueing configurations of up to N patches.
struct CoarseMultiWs {
    float4* pos = nullptr;
    float* zf = nullptr;
    double* partial = nullptr;
    size_t cap_n = 0, cap_part = 0;
    CoarseMultiWs() = default;
    CoarseMultiWs(const CoarseMultiWs&) = delete;
    CoarseMultiWs& operator=(const CoarseMultiWs&) = delete;
    ~CoarseMultiWs();
    void reserve(int N);
};
// As coarse_multi, only enqueued (no allocation, no synchronization).
void coarse_multi_enqueue(hipStream_t s, int problem, int N, const double* frames_dev, const double* Z, double* S,
                          CoarseMultiWs& ws);

// Host (deflate_basis.cpp): T = I + chi0 Z^T S on the k independent columns;
// M = T^{-1} - I padded to kDefl x kDefl (false if T is singular).
void deflation_coarse_matrix(const std::vector<double>& Z, const std::vector<double>& S, int N, int k, double chi0,
                             std::vector<double>& T);
bool deflation_invert(std::vector<double> T, int k, std::vector<double>& M);
// Host, in parallel over configurations: the bases of ncfg configurations
// (frames fr[c], N[c] patches, rows at Zall + kDefl off[c]; N[c] < nmin gives
// k[c] = 0 and zero rows), and M_c = T_c^{-1} - I of each from its coarse
// products Sall (same layout) into Mall (ncfg x kDefl x kDefl); the latter
// leaves configurations with a singular T undeflated (M = 0) and returns
// their count.
void deflation_bases(int ncfg, const double* const* fr, const int* N, const int64_t* off, int nmin, double* Zall,
                     int* k);
int deflation_inverses(int ncfg, const int* N, const int64_t* off, const int* k, const double* chi0,
                       const double* Zall, const double* Sall, double* Mall);

}  // namespace nce
