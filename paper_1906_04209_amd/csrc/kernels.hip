// Device kernels: direct Green's function sums and Krylov vector operations.
// gfx950, wave64. (The block applies are in gemm.hip.)
#include "kernels.hpp"
#include "greens.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>

namespace nce {

// ---------------------------------------------------------------------------
// Direct all-pairs sum. One block per target patch i; each thread owns NPT of
// its K* Zernike nodes (positions relative to c_i kept in registers). For every
// source patch j the block stages j's p skeleton points, relative to c_i, and
// its strengths rho_j in LDS (structure of arrays). Relative positions are
// formed as (c_j - c_i) [FP64, then rounded] + local offsets, so the FP32
// variant keeps full relative accuracy of the short near-field distances.
template <int PROB, int NPT>
__global__ __launch_bounds__(256) void k_direct64(int N, int Kstar, int p, const double* __restrict__ frames,
                                                  const double* __restrict__ node_off,
                                                  const double* __restrict__ skel_off,
                                                  const double* __restrict__ rho, int ldr, double* __restrict__ U,
                                                  const int64_t* __restrict__ lptr, const int* __restrict__ lsrc,
                                                  const int* __restrict__ pt_cfg, const int* __restrict__ live,
                                                  const LogEntry* __restrict__ logtab, TypeTabs tt) {
    extern __shared__ double4 sm64[];  // p source points (x, y, z, rho), half-scaled
    __shared__ LogEntry ltab[kLogTab];
    const int i = blockIdx.x;
    if (live && !live[pt_cfg[i]]) return;
    for (int k = threadIdx.x; k < kLogTab; k += blockDim.x) ltab[k] = logtab[k];
    if (tt.ptype) node_off += (int64_t)tt.ptype[i] * tt.node_stride;
    const double* fi = frames + 9 * (int64_t)i;
    const double cix = fi[0], ciy = fi[1], ciz = fi[2];
    double zx[NPT], zy[NPT], zz[NPT], acc[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int q = threadIdx.x + r * blockDim.x;
        acc[r] = 0.0;
        if (q < Kstar) {
            const double o0 = node_off[3 * q], o1 = node_off[3 * q + 1], o2 = node_off[3 * q + 2];
            zx[r] = 0.5 * (o0 * cix + o1 * fi[3] + o2 * fi[6]);
            zy[r] = 0.5 * (o0 * ciy + o1 * fi[4] + o2 * fi[7]);
            zz[r] = 0.5 * (o0 * ciz + o1 * fi[5] + o2 * fi[8]);
        } else {
            zx[r] = zy[r] = zz[r] = 0.0;
        }
    }
    // sources: every other patch, or the CSR list of patch i
    const int64_t q0 = lptr ? lptr[i] : 0, q1 = lptr ? lptr[i + 1] : N;
    for (int64_t qq = q0; qq < q1; ++qq) {
        const int j = lptr ? lsrc[qq] : (int)qq;
        if (j == i) continue;
        const double* fj = frames + 9 * (int64_t)j;
        const double dcx = fj[0] - cix, dcy = fj[1] - ciy, dcz = fj[2] - ciz;
        // the source's base skeleton (its own radius's with several radii)
        int pj = p, col = 0;
        const double* so = skel_off;
        if (tt.ptype) {
            const int b = tt.ptype[j] * tt.ntab;
            pj = tt.t_p[b];
            col = tt.t_col[b];
            so = skel_off + 3 * (int64_t)tt.t_soff[b];
        }
        __syncthreads();
        for (int m = threadIdx.x; m < pj; m += blockDim.x) {
            const double o0 = so[3 * m], o1 = so[3 * m + 1], o2 = so[3 * m + 2];
            double4 v;
            v.x = 0.5 * (dcx + (o0 * fj[0] + o1 * fj[3] + o2 * fj[6]));
            v.y = 0.5 * (dcy + (o0 * fj[1] + o1 * fj[4] + o2 * fj[7]));
            v.z = 0.5 * (dcz + (o0 * fj[2] + o1 * fj[5] + o2 * fj[8]));
            v.w = rho[(int64_t)j * ldr + col + m];
            sm64[m] = v;
        }
        __syncthreads();
        for (int m = 0; m < pj; ++m) {
            const double4 a = sm64[m];
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const double dx = zx[r] - a.x, dy = zy[r] - a.y, dz = zz[r] - a.z;
                acc[r] += green64_half<PROB>(dx * dx + dy * dy + dz * dz, ltab) * a.w;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int q = threadIdx.x + r * blockDim.x;
        if (q < Kstar) U[(int64_t)i * Kstar + q] = acc[r];
    }
}

template <int PROB, int NPT>
__global__ __launch_bounds__(256) void k_direct32(int N, int Kstar, int p, const double* __restrict__ frames,
                                                  const float* __restrict__ node_off,
                                                  const float* __restrict__ skel_off,
                                                  const float* __restrict__ rho, int ldr, float* __restrict__ U,
                                                  const int64_t* __restrict__ lptr, const int* __restrict__ lsrc,
                                                  const int* __restrict__ pt_cfg, const int* __restrict__ live,
                                                  const LogEntry* __restrict__ logtab, TypeTabs tt) {
    extern __shared__ float4 sm32[];  // p source points (x, y, z, rho), half-scaled
    const int i = blockIdx.x;
    if (live && !live[pt_cfg[i]]) return;
    if (tt.ptype) node_off += (int64_t)tt.ptype[i] * tt.node_stride;
    const double* fi = frames + 9 * (int64_t)i;
    const double cix = fi[0], ciy = fi[1], ciz = fi[2];
    float zx[NPT], zy[NPT], zz[NPT];
    double acc[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int q = threadIdx.x + r * blockDim.x;
        acc[r] = 0.0;
        if (q < Kstar) {
            const float o0 = node_off[3 * q], o1 = node_off[3 * q + 1], o2 = node_off[3 * q + 2];
            zx[r] = 0.5f * (o0 * (float)cix + o1 * (float)fi[3] + o2 * (float)fi[6]);
            zy[r] = 0.5f * (o0 * (float)ciy + o1 * (float)fi[4] + o2 * (float)fi[7]);
            zz[r] = 0.5f * (o0 * (float)ciz + o1 * (float)fi[5] + o2 * (float)fi[8]);
        } else {
            zx[r] = zy[r] = zz[r] = 0.0f;
        }
    }
    constexpr float kLn2 = 0.69314718055994530942f;
    // sources: every other patch, or the CSR list of patch i
    const int64_t q0 = lptr ? lptr[i] : 0, q1 = lptr ? lptr[i + 1] : N;
    for (int64_t qq = q0; qq < q1; ++qq) {
        const int j = lptr ? lsrc[qq] : (int)qq;
        if (j == i) continue;
        const double* fj = frames + 9 * (int64_t)j;
        const float dcx = (float)(fj[0] - cix), dcy = (float)(fj[1] - ciy), dcz = (float)(fj[2] - ciz);
        int pj = p, col = 0;
        const float* so = skel_off;
        if (tt.ptype) {
            const int b = tt.ptype[j] * tt.ntab;
            pj = tt.t_p[b];
            col = tt.t_col[b];
            so = skel_off + 3 * (int64_t)tt.t_soff[b];
        }
        __syncthreads();
        for (int m = threadIdx.x; m < pj; m += blockDim.x) {
            const float o0 = so[3 * m], o1 = so[3 * m + 1], o2 = so[3 * m + 2];
            float4 v;
            v.x = 0.5f * (dcx + (o0 * (float)fj[0] + o1 * (float)fj[3] + o2 * (float)fj[6]));
            v.y = 0.5f * (dcy + (o0 * (float)fj[1] + o1 * (float)fj[4] + o2 * (float)fj[7]));
            v.z = 0.5f * (dcz + (o0 * (float)fj[2] + o1 * (float)fj[5] + o2 * (float)fj[8]));
            v.w = rho[(int64_t)j * ldr + col + m];
            sm32[m] = v;
        }
        __syncthreads();
        float aw[NPT], al[NPT];
#pragma unroll
        for (int r = 0; r < NPT; ++r) aw[r] = al[r] = 0.0f;
        for (int m = 0; m < pj; ++m) {
            const float4 a = sm32[m];
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const float dx = zx[r] - a.x, dy = zy[r] - a.y, dz = zz[r] - a.z;
                float w, l2;
                green32_parts_half<PROB>(dx * dx + dy * dy + dz * dz, w, l2);
                aw[r] += w * a.w;
                al[r] += l2 * a.w;
            }
        }
        // per-source-patch partial sums are short; carry the running total in FP64
#pragma unroll
        for (int r = 0; r < NPT; ++r) acc[r] += (double)(aw[r] - kLn2 * al[r]);
    }
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int q = threadIdx.x + r * blockDim.x;
        if (q < Kstar) U[(int64_t)i * Kstar + q] = (float)acc[r];
    }
}

template <>
hipError_t list_sum<double>(hipStream_t s, int problem, int N, int Kstar, int p, const double* frames,
                            const double* node_off, const double* skel_off, const double* rho, int ldr, double* U,
                            const int64_t* lptr, const int* lsrc, const LogEntry* logtab, const int* pt_cfg,
                            const int* live, const TypeTabs& tt) {
    const size_t sh = 4 * sizeof(double) * (size_t)p;
    if (Kstar > 4 * 256) return hipErrorInvalidValue;
    // nodes per thread: 2 covers K* <= 512 without idle accumulators
    if (Kstar <= 2 * 256) {
        if (problem == 1)
            hipLaunchKernelGGL((k_direct64<1, 2>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
        else
            hipLaunchKernelGGL((k_direct64<0, 2>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
    } else {
        if (problem == 1)
            hipLaunchKernelGGL((k_direct64<1, 4>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
        else
            hipLaunchKernelGGL((k_direct64<0, 4>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
    }
    return hipGetLastError();
}

template <>
hipError_t list_sum<float>(hipStream_t s, int problem, int N, int Kstar, int p, const double* frames,
                            const float* node_off, const float* skel_off, const float* rho, int ldr, float* U,
                            const int64_t* lptr, const int* lsrc, const LogEntry* logtab, const int* pt_cfg,
                            const int* live, const TypeTabs& tt) {
    const size_t sh = 4 * sizeof(float) * (size_t)p;
    if (Kstar > 4 * 256) return hipErrorInvalidValue;
    // nodes per thread: 2 covers K* <= 512 without idle accumulators
    if (Kstar <= 2 * 256) {
        if (problem == 1)
            hipLaunchKernelGGL((k_direct32<1, 2>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
        else
            hipLaunchKernelGGL((k_direct32<0, 2>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
    } else {
        if (problem == 1)
            hipLaunchKernelGGL((k_direct32<1, 4>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
        else
            hipLaunchKernelGGL((k_direct32<0, 4>), dim3(N), dim3(256), sh, s, N, Kstar, p, frames, node_off, skel_off,
                               rho, ldr, U, lptr, lsrc, pt_cfg, live, logtab, tt);
    }
    return hipGetLastError();
}

template <class T>
hipError_t direct_sum(hipStream_t s, int problem, int N, int Kstar, int p, const double* frames, const T* node_off,
                      const T* skel_off, const T* rho, T* U, const LogEntry* logtab, const TypeTabs& tt, int ldr) {
    return list_sum<T>(s, problem, N, Kstar, p, frames, node_off, skel_off, rho, tt.ptype ? ldr : p, U, nullptr,
                       nullptr, logtab, nullptr, nullptr, tt);
}
template hipError_t direct_sum<double>(hipStream_t, int, int, int, int, const double*, const double*, const double*,
                                       const double*, double*, const LogEntry*, const TypeTabs&, int);
template hipError_t direct_sum<float>(hipStream_t, int, int, int, int, const double*, const float*, const float*,
                                      const float*, float*, const LogEntry*, const TypeTabs&, int);

__global__ void k_permute_rows(int64_t N, int K, const int64_t* __restrict__ perm, const double* __restrict__ src,
                               double* __restrict__ dst, int scatter) {
    const int64_t n = N * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t a = e / K, k = e % K;
        if (scatter) dst[perm[a] * K + k] = src[e];
        else dst[e] = src[perm[a] * K + k];
    }
}

hipError_t permute_rows(hipStream_t s, int64_t N, int K, const int64_t* perm, const double* src, double* dst,
                        int scatter) {
    const int64_t blocks = std::min<int64_t>(4096, (N * K + 255) / 256);
    hipLaunchKernelGGL(k_permute_rows, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, N, K, perm, src,
                       dst, scatter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Krylov vector operations (FP64). Reductions are two-stage and deterministic:
// fixed grid, per-block partial sums, then one block sums the partials.

__device__ __forceinline__ double block_sum(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) t += red[k];
    return t;  // valid in thread 0
}

__global__ __launch_bounds__(256) void k_dots_partial(int64_t n, const double* __restrict__ V, int64_t ldv,
                                                      const double* __restrict__ w, double* __restrict__ partial) {
    __shared__ double red[4];
    const int j = blockIdx.y;
    const double* v = V + (int64_t)j * ldv;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        acc += v[e] * w[e];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = t;
}

__global__ __launch_bounds__(256) void k_sum_partials(int nb, const double* __restrict__ partial,
                                                      double* __restrict__ out) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partial[(int64_t)j * nb + b];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0) out[j] = t;
}

static int reduce_blocks(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b < kReduceBlocks ? (b < 1 ? 1 : b) : kReduceBlocks);
}

hipError_t dots(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* w, double* partial,
                double* out) {
    const int nb = reduce_blocks(n);
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, nv), dim3(256), 0, s, n, V, ldv, w, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(nv), dim3(256), 0, s, nb, partial, out);
    return hipGetLastError();
}

hipError_t nrm2(hipStream_t s, int64_t n, const double* x, double* partial, double* out) {
    // out = x . x (the caller takes the square root)
    return dots(s, n, 1, x, n, x, partial, out);
}

__global__ __launch_bounds__(256) void k_axpys(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                               const double* __restrict__ h, double* __restrict__ w) {
    extern __shared__ double hs[];
    for (int j = threadIdx.x; j < nv; j += blockDim.x) hs[j] = h[j];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = w[e];
        for (int j = 0; j < nv; ++j) acc -= hs[j] * V[(int64_t)j * ldv + e];
        w[e] = acc;
    }
}

hipError_t axpys(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* h, double* w) {
    const int64_t nb = (n + 255) / 256;
    const int grid = (int)(nb < 8192 ? nb : 8192);
    hipLaunchKernelGGL(k_axpys, dim3(grid), dim3(256), nv * sizeof(double), s, n, nv, V, ldv, h, w);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_combine(int64_t n, int nv, const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ c, double* __restrict__ x) {
    extern __shared__ double cs[];
    for (int j = threadIdx.x; j < nv; j += blockDim.x) cs[j] = c[j];
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        double acc = x[e];
        for (int j = 0; j < nv; ++j) acc += cs[j] * V[(int64_t)j * ldv + e];
        x[e] = acc;
    }
}

hipError_t combine(hipStream_t s, int64_t n, int nv, const double* V, int64_t ldv, const double* c, double* x) {
    const int64_t nb = (n + 255) / 256;
    const int grid = (int)(nb < 8192 ? nb : 8192);
    hipLaunchKernelGGL(k_combine, dim3(grid), dim3(256), nv * sizeof(double), s, n, nv, V, ldv, c, x);
    return hipGetLastError();
}

__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e];
}
__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = a * x[e] + b * y[e];
}
__global__ void k_cast(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = (float)x[e];
}
__global__ void k_cast_up(int64_t n, const float* __restrict__ x, double* __restrict__ y) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        y[e] = (double)x[e];
}
__global__ void k_rows_scale(int64_t N, int K, const double* __restrict__ a, const float* __restrict__ m,
                             double* __restrict__ x) {
    const int64_t n = N * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / K;
        const int k = (int)(e - i * K);
        x[e] = m ? a[i] * (double)m[e] : (k == 0 ? a[i] : 0.0);
    }
}

__global__ void k_fill(int64_t n, double v, double* __restrict__ x) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = v;
}

static dim3 ew_grid(int64_t n) {
    int64_t nb = (n + 255) / 256;
    return dim3((unsigned)(nb < 16384 ? (nb < 1 ? 1 : nb) : 16384));
}

hipError_t scale_copy(hipStream_t s, int64_t n, double a, const double* x, double* y) {
    hipLaunchKernelGGL(k_scale_copy, ew_grid(n), dim3(256), 0, s, n, a, x, y);
    return hipGetLastError();
}
hipError_t axpby(hipStream_t s, int64_t n, double a, const double* x, double b, double* y) {
    hipLaunchKernelGGL(k_axpby, ew_grid(n), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}
hipError_t cast_d2f(hipStream_t s, int64_t n, const double* x, float* y) {
    hipLaunchKernelGGL(k_cast, ew_grid(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}
hipError_t cast_f2d(hipStream_t s, int64_t n, const float* x, double* y) {
    hipLaunchKernelGGL(k_cast_up, ew_grid(n), dim3(256), 0, s, n, x, y);
    return hipGetLastError();
}
hipError_t rows_scale(hipStream_t s, int64_t N, int K, const double* a, const float* m, double* x) {
    const int64_t n = N * K;
    const int64_t b = (n + 255) / 256;
    hipLaunchKernelGGL(k_rows_scale, dim3((unsigned)(b < 8192 ? (b < 1 ? 1 : b) : 8192)), dim3(256), 0, s, N, K, a, m,
                       x);
    return hipGetLastError();
}

hipError_t fill(hipStream_t s, int64_t n, double v, double* x) {
    hipLaunchKernelGGL(k_fill, ew_grid(n), dim3(256), 0, s, n, v, x);
    return hipGetLastError();
}

__global__ void k_unit_rhs(int64_t n, int K, double* __restrict__ b) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        b[e] = e % K == 0 ? 1.0 : 0.0;
}

hipError_t unit_rhs(hipStream_t s, int64_t N, int K, double* b) {
    const int64_t n = N * K;
    hipLaunchKernelGGL(k_unit_rhs, ew_grid(n), dim3(256), 0, s, n, K, b);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_flux(int N, int K, const double* __restrict__ I, const double* __restrict__ x,
                                              double* __restrict__ flux, double* __restrict__ partial) {
    __shared__ double red[4];
    double mine = 0.0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        double f = 0.0;
        for (int k = 0; k < K; ++k) f += I[k] * x[(int64_t)i * K + k];
        if (flux) flux[i] = f;
        mine += f;
    }
    const double t = block_sum(mine, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

hipError_t patch_flux(hipStream_t s, int N, int K, const double* I, const double* x, double* flux, double* partial,
                      double* sum) {
    const int nb = reduce_blocks(N);
    hipLaunchKernelGGL(k_flux, dim3(nb), dim3(256), 0, s, N, K, I, x, flux, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, nb, partial, sum);
    return hipGetLastError();
}

}  // namespace nce
