// Coarse-space deflation of the FP32 inner solves: basis, coarse operator on
// it, and the preconditioner apply (see deflate.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>
#include <vector>

#include "deflate.hpp"
#include "greens.hpp"
#include "kernels.hpp"

namespace nce {

namespace {

constexpr int kMTile = 256;   // source centres per LDS tile
constexpr int kDotBlocks = 256;

void chk(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

// pos[j] = c_j / 2; zf[j] = Z_j in FP32
__global__ void k_defl_src(int N, const double* __restrict__ frames, const double* __restrict__ Z,
                           float4* __restrict__ pos, float* __restrict__ zf) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const double* f = frames + 9 * (int64_t)j;
    pos[j] = make_float4((float)(0.5 * f[0]), (float)(0.5 * f[1]), (float)(0.5 * f[2]), 0.0f);
#pragma unroll
    for (int q = 0; q < kDefl; ++q) zf[(int64_t)j * kDefl + q] = (float)Z[(int64_t)j * kDefl + q];
}

// partial[split][i][q] = sum over this split's sources j != i of G(c_i, c_j) Z_j[q]
template <int PROB>
__global__ __launch_bounds__(256) void k_coarse_multi(int N, const float4* __restrict__ pos,
                                                      const float* __restrict__ zf, int chunk,
                                                      double* __restrict__ partial) {
    __shared__ float4 tp[kMTile];
    __shared__ float4 tz[kMTile][kDefl / 4];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const float4 ci = pos[i < N ? i : N - 1];
    double acc[kDefl];
#pragma unroll
    for (int q = 0; q < kDefl; ++q) acc[q] = 0.0;
    const int j0 = blockIdx.y * chunk, j1 = min(N, j0 + chunk);
    constexpr float kLn2 = 0.69314718055994530942f;
    const float4* z4 = reinterpret_cast<const float4*>(zf);
    for (int t0 = j0; t0 < j1; t0 += kMTile) {
        const int tl = min(kMTile, j1 - t0);
        __syncthreads();
        for (int k = threadIdx.x; k < tl; k += blockDim.x) {
            tp[k] = pos[t0 + k];
#pragma unroll
            for (int qq = 0; qq < kDefl / 4; ++qq) tz[k][qq] = z4[(int64_t)(t0 + k) * (kDefl / 4) + qq];
        }
        __syncthreads();
        float a[kDefl];
#pragma unroll
        for (int q = 0; q < kDefl; ++q) a[q] = 0.0f;
        for (int k = 0; k < tl; ++k) {
            const float4 s = tp[k];
            const float dx = ci.x - s.x, dy = ci.y - s.y, dz = ci.z - s.z;
            const float h2 = dx * dx + dy * dy + dz * dz;
            // the target itself (h2 = 0) contributes nothing
            const bool self = !(h2 > 0.0f);
            float w, l2;
            green32_parts_half<PROB>(self ? 1.0f : h2, w, l2);
            const float g = self ? 0.0f : w - kLn2 * l2;
#pragma unroll
            for (int qq = 0; qq < kDefl / 4; ++qq) {
                const float4 z = tz[k][qq];
                a[4 * qq] += g * z.x;
                a[4 * qq + 1] += g * z.y;
                a[4 * qq + 2] += g * z.z;
                a[4 * qq + 3] += g * z.w;
            }
        }
#pragma unroll
        for (int q = 0; q < kDefl; ++q) acc[q] += (double)a[q];
    }
    if (i < N)
#pragma unroll
        for (int q = 0; q < kDefl; ++q) partial[((int64_t)blockIdx.y * N + i) * kDefl + q] = acc[q];
}

__global__ void k_sum_splits(int64_t n, int nsplit, const double* __restrict__ partial, double* __restrict__ S) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    double v = 0.0;
    for (int k = 0; k < nsplit; ++k) v += partial[(int64_t)k * n + e];
    S[e] = v;
}

// partial[b][q] = sum over this block's patches i of Z[i][q] v[i][0]
__global__ __launch_bounds__(256) void k_defl_dots(int N, int K, const double* __restrict__ Z,
                                                   const double* __restrict__ v, double* __restrict__ partial) {
    __shared__ double red[kDefl][256];
    double acc[kDefl];
#pragma unroll
    for (int q = 0; q < kDefl; ++q) acc[q] = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const double x = v[(int64_t)i * K];
#pragma unroll
        for (int q = 0; q < kDefl; ++q) acc[q] += Z[(int64_t)i * kDefl + q] * x;
    }
#pragma unroll
    for (int q = 0; q < kDefl; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < kDefl; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kDefl) partial[blockIdx.x * kDefl + threadIdx.x] = red[threadIdx.x][0];
}

// out[i][0] += sum_q Z[i][q] c[q], c = Minv (sum_b partial[b]) (every block
// forms c itself, in a fixed order)
__global__ __launch_bounds__(256) void k_defl_update(int N, int K, const double* __restrict__ Z,
                                                     const double* __restrict__ Minv, const double* __restrict__ partial,
                                                     int nb, double* __restrict__ out) {
    __shared__ double red[kDefl][256];
    __shared__ double zt[kDefl], c[kDefl];
    // sum of the nb <= 256 block partials: one row per thread, then a tree in
    // LDS (the same order in every block)
#pragma unroll
    for (int q = 0; q < kDefl; ++q)
        red[q][threadIdx.x] = (int)threadIdx.x < nb ? partial[threadIdx.x * kDefl + q] : 0.0;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < kDefl; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kDefl) zt[threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
    if (threadIdx.x < kDefl) {
        double s = 0.0;
        for (int r = 0; r < kDefl; ++r) s += Minv[threadIdx.x * kDefl + r] * zt[r];
        c[threadIdx.x] = s;
    }
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kDefl; ++q) s += Z[(int64_t)i * kDefl + q] * c[q];
        out[(int64_t)i * K] += s;
    }
}

// Batched form, one block per configuration c (patches [pseg[c], pseg[c + 1])):
// d[c] = M_c Z_c^T v[:, 0]; inactive configurations get d[c] = 0.
__global__ __launch_bounds__(256) void k_bdefl_dots(int K, const int64_t* __restrict__ pseg,
                                                    const double* __restrict__ Z, const double* __restrict__ M,
                                                    const int* __restrict__ active, const double* __restrict__ v,
                                                    double* __restrict__ d) {
    __shared__ double red[kDefl][256];
    __shared__ double c[kDefl];
    const int cf = blockIdx.x;
    const bool on = !active || active[cf];
    const int64_t p0 = pseg[cf], p1 = pseg[cf + 1];
    double acc[kDefl];
#pragma unroll
    for (int q = 0; q < kDefl; ++q) acc[q] = 0.0;
    if (on)
        for (int64_t i = p0 + threadIdx.x; i < p1; i += blockDim.x) {
            const double x = v[i * K];
#pragma unroll
            for (int q = 0; q < kDefl; ++q) acc[q] += Z[i * kDefl + q] * x;
        }
#pragma unroll
    for (int q = 0; q < kDefl; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
#pragma unroll
            for (int q = 0; q < kDefl; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < kDefl) c[threadIdx.x] = red[threadIdx.x][0];
    __syncthreads();
    if (threadIdx.x < kDefl) {
        const double* Mc = M + (int64_t)cf * kDefl * kDefl + threadIdx.x * kDefl;
        double s = 0.0;
        for (int r = 0; r < kDefl; ++r) s += Mc[r] * c[r];
        d[(int64_t)cf * kDefl + threadIdx.x] = on ? s : 0.0;
    }
}

// v[i][0] += sum_q Z[i][q] d[cfg(i)][q] for every patch i
__global__ __launch_bounds__(256) void k_bdefl_update(int64_t npatch, int K, const int* __restrict__ patch_cfg,
                                                      const double* __restrict__ Z, const double* __restrict__ d,
                                                      double* __restrict__ v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npatch) return;
    const double* dc = d + (int64_t)patch_cfg[i] * kDefl;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < kDefl; ++q) s += Z[i * kDefl + q] * dc[q];
    v[i * K] += s;
}

}  // namespace

CoarseMultiWs::~CoarseMultiWs() {
    for (void* p : {(void*)pos, (void*)zf, (void*)partial})
        if (p) (void)hipFree(p);
}

namespace {
int coarse_splits(int N) {
    const int ntb = (N + 255) / 256;
    return std::max(1, std::min((N + kMTile - 1) / kMTile, (2048 + ntb - 1) / ntb));
}
}  // namespace

void CoarseMultiWs::reserve(int N) {
    const size_t np = (size_t)N, npart = (size_t)coarse_splits(N) * N * kDefl;
    if (np > cap_n) {
        if (pos) (void)hipFree(pos);
        if (zf) (void)hipFree(zf);
        pos = nullptr;
        zf = nullptr;
        cap_n = 0;
        chk(hipMalloc((void**)&pos, sizeof(float4) * np), "hipMalloc");
        chk(hipMalloc((void**)&zf, sizeof(float) * np * kDefl), "hipMalloc");
        cap_n = np;
    }
    if (npart > cap_part) {
        if (partial) (void)hipFree(partial);
        partial = nullptr;
        cap_part = 0;
        chk(hipMalloc((void**)&partial, sizeof(double) * npart), "hipMalloc");
        cap_part = npart;
    }
}

void coarse_multi_enqueue(hipStream_t s, int problem, int N, const double* frames_dev, const double* Z, double* S,
                          CoarseMultiWs& ws) {
    const int ntb = (N + 255) / 256;
    const int nsplit = coarse_splits(N);
    const int chunk = (N + nsplit - 1) / nsplit;
    if ((size_t)N > ws.cap_n || (size_t)nsplit * N * kDefl > ws.cap_part)
        throw std::runtime_error("coarse_multi workspace too small");
    hipLaunchKernelGGL(k_defl_src, dim3(ntb), dim3(256), 0, s, N, frames_dev, Z, ws.pos, ws.zf);
    if (problem == 1)
        hipLaunchKernelGGL(k_coarse_multi<1>, dim3(ntb, nsplit), dim3(256), 0, s, N, ws.pos, ws.zf, chunk, ws.partial);
    else
        hipLaunchKernelGGL(k_coarse_multi<0>, dim3(ntb, nsplit), dim3(256), 0, s, N, ws.pos, ws.zf, chunk, ws.partial);
    const int64_t n = (int64_t)N * kDefl;
    hipLaunchKernelGGL(k_sum_splits, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nsplit, ws.partial, S);
    chk(hipGetLastError(), "coarse_multi");
}

void coarse_multi(hipStream_t s, int problem, int N, const double* frames_dev, const double* Z, double* S) {
    CoarseMultiWs ws;
    ws.reserve(N);
    coarse_multi_enqueue(s, problem, N, frames_dev, Z, S, ws);
    chk(hipStreamSynchronize(s), "sync");
}

Deflation::~Deflation() {
    for (void* p : {(void*)Z, (void*)Minv, (void*)partial})
        if (p) (void)hipFree(p);
}

int deflation_member(hipStream_t s, int N, int problem, double chi0, const std::vector<double>& frames,
                     const double* frames_dev, std::vector<double>& Zh, std::vector<double>& M,
                     std::vector<double>* Tout, const std::vector<double>* chi_patch) {
    if (chi_patch && chi_patch->size() != (size_t)N)
        throw std::runtime_error("deflation: one charge per patch");
    M.assign((size_t)kDefl * kDefl, 0.0);
    if (N < kDeflMinN) {
        Zh.assign((size_t)N * kDefl, 0.0);
        if (Tout) Tout->clear();
        return 0;
    }
    const int k = deflation_basis(frames, N, Zh);
    double* Zd = nullptr;
    double* Sd = nullptr;
    chk(hipMalloc((void**)&Zd, sizeof(double) * Zh.size()), "hipMalloc");
    if (hipMalloc((void**)&Sd, sizeof(double) * Zh.size()) != hipSuccess) {
        (void)hipFree(Zd);
        throw std::runtime_error("hipMalloc failed");
    }
    std::vector<double> Sh(Zh.size());
    try {
        // the sources of the pass: Z, or D Z with D = diag(chi0_j) for per-patch charges
        std::vector<double> Zs;
        if (chi_patch) {
            Zs = Zh;
            for (int j = 0; j < N; ++j)
                for (int q = 0; q < kDefl; ++q) Zs[(size_t)j * kDefl + q] *= (*chi_patch)[j];
        }
        const std::vector<double>& src = chi_patch ? Zs : Zh;
        chk(hipMemcpyAsync(Zd, src.data(), sizeof(double) * src.size(), hipMemcpyHostToDevice, s), "copy");
        coarse_multi(s, problem, N, frames_dev, Zd, Sd);
        chk(hipMemcpy(Sh.data(), Sd, sizeof(double) * Sh.size(), hipMemcpyDeviceToHost), "copy");
    } catch (...) {
        (void)hipFree(Zd);
        (void)hipFree(Sd);
        throw;
    }
    (void)hipFree(Zd);
    (void)hipFree(Sd);
    // T = Z^T (I + chi0 G) Z on the k independent columns (Z^T Z = I); with
    // per-patch charges T = Z^T (I + G D) Z, S already holding G D Z
    std::vector<double> T;
    deflation_coarse_matrix(Zh, Sh, N, k, chi_patch ? 1.0 : chi0, T);
    if (Tout) *Tout = T;
    // a singular T (not met in practice) leaves the configuration undeflated:
    // M = 0 makes M^{-1} the identity
    if (!deflation_invert(T, k, M)) {
        M.assign((size_t)kDefl * kDefl, 0.0);
        return 0;
    }
    return k;
}

void Deflation::build(hipStream_t s, int N_, int K_, int problem, double chi0, const std::vector<double>& frames,
                      const double* frames_dev, const std::vector<double>* chi_patch) {
    N = N_;
    K = K_;
    std::vector<double> Zh, M;
    k = deflation_member(s, N, problem, chi0, frames, frames_dev, Zh, M, &T, chi_patch);
    chk(hipMalloc((void**)&Z, sizeof(double) * Zh.size()), "hipMalloc");
    chk(hipMalloc((void**)&Minv, sizeof(double) * kDefl * kDefl), "hipMalloc");
    chk(hipMalloc((void**)&partial, sizeof(double) * kDotBlocks * kDefl), "hipMalloc");
    chk(hipMemcpyAsync(Z, Zh.data(), sizeof(double) * Zh.size(), hipMemcpyHostToDevice, s), "copy");
    chk(hipMemcpyAsync(Minv, M.data(), sizeof(double) * M.size(), hipMemcpyHostToDevice, s), "copy");
    chk(hipStreamSynchronize(s), "sync");
}

hipError_t Deflation::apply_stride(hipStream_t s, const double* in, double* out, int stride) const {
    if (out != in) {
        const hipError_t e = hipMemcpyAsync(out, in, sizeof(double) * (size_t)N * stride, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    const int nb = std::max(1, std::min(kDotBlocks, (N + 255) / 256));
    hipLaunchKernelGGL(k_defl_dots, dim3(nb), dim3(256), 0, s, N, stride, Z, in, partial);
    const int nu = std::max(1, std::min(1024, (N + 255) / 256));
    hipLaunchKernelGGL(k_defl_update, dim3(nu), dim3(256), 0, s, N, stride, Z, Minv, partial, nb, out);
    return hipGetLastError();
}

hipError_t deflation_apply_batched(hipStream_t s, int ncfg, int64_t npatch, int K, const int64_t* pseg,
                                   const int* patch_cfg, const double* Z, const double* M, const int* active,
                                   double* d, double* v) {
    if (ncfg <= 0 || npatch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bdefl_dots, dim3(ncfg), dim3(256), 0, s, K, pseg, Z, M, active, v, d);
    hipLaunchKernelGGL(k_bdefl_update, dim3((unsigned)((npatch + 255) / 256)), dim3(256), 0, s, npatch, K, patch_cfg,
                       Z, d, v);
    return hipGetLastError();
}

}  // namespace nce
