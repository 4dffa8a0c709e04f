// Device kernels of the system matrix apply (Section 8, Step 3) and the
// Krylov solver, for gfx950 (wave64). Launch wrappers are host functions that
// enqueue on the given stream and return hipError_t.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "greens.hpp"

namespace nce {

// Green's function of the unit sphere on the surface, as a function of
// w = 2/d (d = chord): exterior w - log(1 + w), interior w + log(w^2/(1 + w)).
// (These are eqs. Gextonsurface / Gintonsurface with the logs combined.)

// C[i][j] = alpha * sum_k A[i][k] B[j][k] + beta * D[i][j]   (row-major, "NT")
// A: m x k (lda), B: n x k (ldb), C/D: m x n (ldc). D may be null (beta ignored).
template <class T>
hipError_t gemm_nt(hipStream_t s, int m, int n, int k, const T* A, int lda, const T* B, int ldb,
                   T* C, int ldc, const double* D, int ldd);

// C[i][j] (+)= alpha sum_k A[i*sai + k*sak] B[k*sbk + j*sbj] on the matrix cores
// (accumulate != 0 adds into C).
template <class T>
hipError_t gemm_strided(hipStream_t s, int m, int n, int k, const T* A, int64_t sai, int64_t sak, const T* B,
                        int64_t sbk, int64_t sbj, T* C, int64_t ldc, T alpha, int accumulate);

// y[i][c] = x[i][c] + sum_q U[i][q] P[c][q]  (FP64 out, U/P in T)
template <class T>
hipError_t p_apply(hipStream_t s, int N, int K, int Kstar, const T* U, const T* P, const double* x,
                   double* y);

// Several patch radii in one configuration: the patch type of every patch and,
// per (type, outgoing table), where its skeleton starts in the concatenated
// skeleton offsets, where its strengths start in a patch's row of rho, and its
// size; each type's sampling-node offsets follow one another (node_stride
// entries apart). ptype == nullptr: one patch radius, the arguments of the
// call itself apply.
struct TypeTabs {
    const int* ptype = nullptr;
    const int* t_soff = nullptr;
    const int* t_col = nullptr;
    const int* t_p = nullptr;
    int ntab = 1;
    int node_stride = 0;
};

// Direct all-pairs incoming field at the Zernike nodes of every patch:
// U[i][q] = sum_{j != i} sum_m G(|z_iq - s_jm|) rho[j][m]
// frames: N x 9 FP64 (c, e1, e2); node_off: Kstar x 3, skel_off: p x 3 local
// offsets in T precision; rho: N x p in T.
// logtab: the FP64 logarithm's table (device, kLogTab entries; unused by FP32).
// With several radii (tt.ptype set) p is the largest base skeleton and ldr the
// row length of rho.
template <class T>
hipError_t direct_sum(hipStream_t s, int problem, int N, int Kstar, int p, const double* frames,
                      const T* node_off, const T* skel_off, const T* rho, T* U, const LogEntry* logtab,
                      const TypeTabs& tt = TypeTabs(), int ldr = 0);

// Same with the sources of target i restricted to lsrc[lptr[i] .. lptr[i+1]) (CSR)
// and the strengths of patch j at rho[j * ldr .. j * ldr + p).
// Targets i with live && !live[pt_cfg[i]] are skipped (pt_cfg, live may be null).
template <class T>
hipError_t list_sum(hipStream_t s, int problem, int N, int Kstar, int p, const double* frames, const T* node_off,
                    const T* skel_off, const T* rho, int ldr, T* U, const int64_t* lptr, const int* lsrc,
                    const LogEntry* logtab, const int* pt_cfg = nullptr, const int* live = nullptr,
                    const TypeTabs& tt = TypeTabs());

// Rows of K values: scatter = 0: dst[a] = src[perm[a]]; scatter = 1: dst[perm[a]] = src[a].
hipError_t permute_rows(hipStream_t s, int64_t N, int K, const int64_t* perm, const double* src, double* dst,
                        int scatter);

// Krylov helpers (FP64).
hipError_t dots(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* w,
                double* partial, double* out);  // out[j] = V_j . w, j < nv
hipError_t axpys(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* h,
                 double* w);                     // w -= sum_j h_j V_j
hipError_t nrm2(hipStream_t s, int64_t n, const double* x, double* partial, double* out);
hipError_t scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y);  // y = a x
hipError_t axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y);  // y = a x + b y
hipError_t combine(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* c,
                   double* x);                   // x += sum_j c_j V_j
hipError_t cast_d2f(hipStream_t s, int64_t n, const double* x, float* y);
hipError_t cast_f2d(hipStream_t s, int64_t n, const float* x, double* y);
hipError_t fill(hipStream_t s, int64_t n, double v, double* x);
// b = e_0 on each of N patches (the right-hand side P 1), N x K
hipError_t unit_rhs(hipStream_t s, int64_t N, int K, double* b);
// x[i][k] = a[i] m[i][k] (m: N x K FP32), or a[i] [k == 0] when m is null
hipError_t rows_scale(hipStream_t s, int64_t N, int K, const double* a, const float* m, double* x);
// flux[i] = sum_k I[k] x[i][k]; total written to *sum (two-stage)
hipError_t patch_flux(hipStream_t s, int N, int K, const double* I, const double* x, double* flux,
                      double* partial, double* sum);

constexpr int kReduceBlocks = 1024;  // partial-sum slots used by the reductions

}  // namespace nce
