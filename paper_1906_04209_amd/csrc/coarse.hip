// Monopole (coarse) model of the multiple-scattering system, used to start
// GMRES near the solution's global part.
//
// Take every patch's unknowns as a multiple of the isolated-patch solution,
// f_i = a_i e_0 (the right-hand side P 1 is e_0), and every far field as a
// point charge at the patch centre: the strengths T f_j then carry the total
// charge chi0 a_j with chi0 = sum_m T[m][0], and P maps the (nearly constant)
// incoming field over patch i to e_0 times its value at c_i. Row 0 of the
// system (eq. opinteqnsdisc) becomes the N x N system
//
//     a_i + chi0 sum_{j != i} G(c_i, c_j) a_j = 1,
//
// whose matrix carries the strong, long-range coupling of many patches that
// makes plain GMRES slow. With patches of several radii the charge is patch
// j's own, chi0_j from its radius's outgoing table, inside the sum (P acts on
// functions of t/eps and is the same for every radius, and so are row 0 and
// the right-hand side e_0). It is solved here by GMRES on the device, with the
// all-pairs sum over centres in FP32 (FP64 accumulation): O(N^2) pair
// evaluations, about a hundredth of one full system apply at N = 1e5.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "coarse.hpp"
#include "greens.hpp"
#include "kernels.hpp"

namespace nce {

namespace {

constexpr int kTile = 1024;  // source centres per LDS tile
constexpr int kTgt = 4;      // target centres per thread

void chk(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// src[j] = (c_j / 2, a_j), or (c_j / 2, chi0_j a_j) with per-patch charges
__global__ void k_coarse_src(int N, const double* __restrict__ frames, const double* __restrict__ a,
                             const double* __restrict__ chi, float4* __restrict__ src) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double* f = frames + 9 * (int64_t)j;
    const double q = chi ? chi[j] * a[j] : a[j];
    src[j] = make_float4((float)(0.5 * f[0]), (float)(0.5 * f[1]), (float)(0.5 * f[2]), (float)q);
}

// partial[split * N + i] = sum over this split's sources j != i of G(c_i, c_j) a_j.
// Block: 256 threads x kTgt targets; blockIdx.y = source split.
template <int PROB>
__global__ __launch_bounds__(256) void k_coarse_sum(int N, const float4* __restrict__ src, int chunk,
                                                    double* __restrict__ partial) {
    __shared__ float4 tile[kTile];
    const int i0 = blockIdx.x * 256 * kTgt;
    float tx[kTgt], ty[kTgt], tz[kTgt];
    double acc[kTgt];
#pragma unroll
    for (int r = 0; r < kTgt; ++r) {
        const int i = i0 + threadIdx.x + 256 * r;
        const float4 c = src[i < N ? i : N - 1];
        tx[r] = c.x;
        ty[r] = c.y;
        tz[r] = c.z;
        acc[r] = 0.0;
    }
    const int j0 = blockIdx.y * chunk, j1 = min(N, j0 + chunk);
    constexpr float kLn2 = 0.69314718055994530942f;
    for (int t0 = j0; t0 < j1; t0 += kTile) {
        const int tl = min(kTile, j1 - t0);
        __syncthreads();
        for (int k = threadIdx.x; k < tl; k += blockDim.x) tile[k] = src[t0 + k];
        __syncthreads();
        float aw[kTgt], al[kTgt];
#pragma unroll
        for (int r = 0; r < kTgt; ++r) aw[r] = al[r] = 0.0f;
        // only a tile that holds some of this block's targets can meet a
        // target itself; every other tile skips the check
        const bool overlap = t0 < i0 + 256 * kTgt && i0 < t0 + tl;
        if (overlap) {
            for (int k = 0; k < tl; ++k) {
                const float4 s = tile[k];
#pragma unroll
                for (int r = 0; r < kTgt; ++r) {
                    const float dx = tx[r] - s.x, dy = ty[r] - s.y, dz = tz[r] - s.z;
                    const float h2 = dx * dx + dy * dy + dz * dz;
                    // the target itself (h2 = 0) contributes nothing
                    const bool self = !(h2 > 0.0f);
                    float w, l2;
                    green32_parts_half<PROB>(self ? 1.0f : h2, w, l2);
                    const float q = self ? 0.0f : s.w;
                    aw[r] += w * q;
                    al[r] += l2 * q;
                }
            }
        } else {
            for (int k = 0; k < tl; ++k) {
                const float4 s = tile[k];
#pragma unroll
                for (int r = 0; r < kTgt; ++r) {
                    const float dx = tx[r] - s.x, dy = ty[r] - s.y, dz = tz[r] - s.z;
                    float w, l2;
                    green32_parts_half<PROB>(dx * dx + dy * dy + dz * dz, w, l2);
                    aw[r] += w * s.w;
                    al[r] += l2 * s.w;
                }
            }
        }
#pragma unroll
        for (int r = 0; r < kTgt; ++r) acc[r] += (double)(aw[r] - kLn2 * al[r]);
    }
#pragma unroll
    for (int r = 0; r < kTgt; ++r) {
        const int i = i0 + threadIdx.x + 256 * r;
        if (i < N) partial[(int64_t)blockIdx.y * N + i] = acc[r];
    }
}

// y_i = a_i + scale sum_split partial[split][i] (scale = chi0, or 1 when the
// sources carry their own charges)
__global__ void k_coarse_finish(int N, int nsplit, const double* __restrict__ partial, const double* __restrict__ a,
                                double scale, double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += partial[(int64_t)k * N + i];
    y[i] = a[i] + scale * s;
}

// q_j = chi0_j a_j (FP32)
__global__ void k_coarse_q32(int N, const double* __restrict__ a, const double* __restrict__ chi, double chi0,
                             float* __restrict__ q) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < N) q[j] = (float)((chi ? chi[j] : chi0) * a[j]);
}

// y_i = a_i + u_i
__global__ void k_coarse_add32(int N, const double* __restrict__ a, const float* __restrict__ u,
                               double* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) y[i] = a[i] + (double)u[i];
}

}  // namespace

hipError_t CoarseSolver::charges32(hipStream_t s, int n, const double* a, float* q) const {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_q32, dim3((n + 255) / 256), dim3(256), 0, s, n, a, chi, chi0, q);
    return hipGetLastError();
}

hipError_t CoarseSolver::finish32(hipStream_t s, int n, const double* a, const float* u, double* y) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(k_coarse_add32, dim3((n + 255) / 256), dim3(256), 0, s, n, a, u, y);
    return hipGetLastError();
}

// source splits for a layout of n centres: enough for >= 2048 blocks, each
// split at least one tile
static int splits_for(int n) {
    const int ntb = (n + 256 * kTgt - 1) / (256 * kTgt);
    return std::max(1, std::min((n + kTile - 1) / kTile, (2048 + ntb - 1) / ntb));
}

CoarseSolver::CoarseSolver(int N_, int problem_, double chi0_, int maxit_)
    : N(N_), problem(problem_), chi0(chi0_), maxit(maxit_) {
    // partial sums for any layout of n <= N centres
    size_t maxpart = 1;
    for (int n = 1; n <= N; ++n) maxpart = std::max(maxpart, (size_t)splits_for(n) * n);
    chk(hipMalloc((void**)&src, sizeof(float4) * (size_t)N), "hipMalloc");
    chk(hipMalloc((void**)&part, sizeof(double) * maxpart), "hipMalloc");
    chk(hipMalloc((void**)&V, sizeof(double) * (size_t)N * (maxit + 1)), "hipMalloc");
    chk(hipMalloc((void**)&h, sizeof(double) * (size_t)(maxit + 2)), "hipMalloc");
    chk(hipMalloc((void**)&rpart, sizeof(double) * (size_t)kReduceBlocks * (maxit + 2)), "hipMalloc");
    chk(hipMalloc((void**)&scal, sizeof(double) * 8), "hipMalloc");
    chk(hipMalloc((void**)&tmp, sizeof(double) * (size_t)N), "hipMalloc");
}

CoarseSolver::~CoarseSolver() {
    for (void* p : {(void*)src, (void*)part, (void*)V, (void*)h, (void*)rpart, (void*)scal, (void*)tmp, (void*)chi})
        if (p) (void)hipFree(p);
}

void CoarseSolver::set_charges(hipStream_t s, const std::vector<double>& chi0_patch) {
    if (chi0_patch.empty() || chi0_patch.size() > (size_t)N)
        throw std::runtime_error("coarse charges: one value per patch of at most N patches");
    if (!chi) chk(hipMalloc((void**)&chi, sizeof(double) * (size_t)N), "hipMalloc");
    chk(hipMemcpyAsync(chi, chi0_patch.data(), sizeof(double) * chi0_patch.size(), hipMemcpyHostToDevice, s), "copy");
    chk(hipStreamSynchronize(s), "sync");
}

void CoarseSolver::apply(hipStream_t s, int n, const double* frames, const double* a, double* y) {
    if (n < 1 || n > N) throw std::runtime_error("coarse apply: layout larger than the solver");
    if (fast_apply && n == N) {
        fast_apply(s, a, y);
        return;
    }
    const int nsplit = splits_for(n), chunk = (n + nsplit - 1) / nsplit;
    hipLaunchKernelGGL(k_coarse_src, dim3((n + 255) / 256), dim3(256), 0, s, n, frames, a, chi, src);
    const dim3 grid((n + 256 * kTgt - 1) / (256 * kTgt), nsplit);
    if (problem == 1)
        hipLaunchKernelGGL(k_coarse_sum<1>, grid, dim3(256), 0, s, n, src, chunk, part);
    else
        hipLaunchKernelGGL(k_coarse_sum<0>, grid, dim3(256), 0, s, n, src, chunk, part);
    hipLaunchKernelGGL(k_coarse_finish, dim3((n + 255) / 256), dim3(256), 0, s, n, nsplit, part, a,
                       chi ? 1.0 : chi0, y);
    chk(hipGetLastError(), "coarse apply");
}

int CoarseSolver::solve(hipStream_t s, int nn, const double* frames, double tol, double* a, const Deflation* defl) {
    // GMRES (CGS2, Givens on the host) for C a = 1 from a = 0; with defl on
    // C M^{-1}, a = M^{-1} V y at the end
    if (nn < 1 || nn > N) throw std::runtime_error("coarse solve: layout larger than the solver");
    if (defl && defl->N != nn) throw std::runtime_error("coarse solve: deflation of another layout");
    const int64_t n = nn;
    std::vector<double> one((size_t)n, 1.0);
    chk(hipMemcpyAsync(V, one.data(), sizeof(double) * n, hipMemcpyHostToDevice, s), "copy");
    const double bnorm = std::sqrt((double)n);
    chk(scale_copy(s, n, 1.0 / bnorm, V, V), "scale");
    chk(fill(s, n, 0.0, a), "fill");
    std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
    std::vector<double> h1(maxit + 1), h2(maxit + 1);
    g[0] = bnorm;
    int k = 0;
    for (k = 0; k < maxit; ++k) {
        double* w = V + (int64_t)(k + 1) * n;
        if (defl) {
            chk(defl->apply_stride(s, V + (int64_t)k * n, tmp, 1), "deflation");
            apply(s, nn, frames, tmp, w);
        } else {
            apply(s, nn, frames, V + (int64_t)k * n, w);
        }
        for (int pass = 0; pass < 2; ++pass) {
            chk(dots(s, n, k + 1, V, n, w, rpart, h), "dots");
            chk(axpys(s, n, k + 1, V, n, h, w), "axpys");
            chk(hipMemcpyAsync(pass == 0 ? h1.data() : h2.data(), h, sizeof(double) * (k + 1),
                               hipMemcpyDeviceToHost, s),
                "copy");
        }
        chk(dots(s, n, 1, w, n, w, rpart, scal), "dots");
        double hk1sq = 0;
        chk(hipMemcpyAsync(&hk1sq, scal, sizeof(double), hipMemcpyDeviceToHost, s), "copy");
        chk(hipStreamSynchronize(s), "sync");
        const double hk1 = std::sqrt(std::max(hk1sq, 0.0));
        if (!std::isfinite(hk1)) throw std::runtime_error("non-finite coarse Arnoldi norm");
        for (int j = 0; j <= k; ++j) H[(size_t)j * maxit + k] = h1[j] + h2[j];
        H[(size_t)(k + 1) * maxit + k] = hk1;
        for (int j = 0; j < k; ++j) {
            const double x = H[(size_t)j * maxit + k], y = H[(size_t)(j + 1) * maxit + k];
            H[(size_t)j * maxit + k] = cs[j] * x + sn[j] * y;
            H[(size_t)(j + 1) * maxit + k] = -sn[j] * x + cs[j] * y;
        }
        const double x = H[(size_t)k * maxit + k];
        const double den = std::hypot(x, hk1);
        cs[k] = x / den;
        sn[k] = hk1 / den;
        H[(size_t)k * maxit + k] = den;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        if (std::fabs(g[k + 1]) <= tol * bnorm || hk1 <= 1e-14 * bnorm) {
            ++k;
            break;
        }
        chk(scale_copy(s, n, 1.0 / hk1, w, w), "scale");
    }
    const int m = std::min(k, maxit);
    std::vector<double> y(m);
    for (int i = m - 1; i >= 0; --i) {
        double acc = g[i];
        for (int j = i + 1; j < m; ++j) acc -= H[(size_t)i * maxit + j] * y[j];
        y[i] = acc / H[(size_t)i * maxit + i];
    }
    chk(hipMemcpyAsync(h, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s), "copy");
    chk(combine(s, n, m, V, n, h, a), "combine");
    if (defl) chk(defl->apply_stride(s, a, a, 1), "deflation");
    chk(hipStreamSynchronize(s), "sync");
    return m;
}

}  // namespace nce
