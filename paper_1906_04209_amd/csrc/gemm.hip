// Dense matrix products on the matrix cores (CDNA MFMA), FP64 and FP32.
//
// C[i][j] (=|+=) alpha * sum_k A(i,k) B(k,j) (+ D[i][j]), with arbitrary
// element strides A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], so
// one kernel serves the NT products of the block applies (rho = f T^T and
// y = f + U P^T, Section 8 Step 3 items 1 and 5) and the NN / TN products of
// the warm-start network's forward and backward passes.
//
// Block: 256 threads = 4 waves over a 64 x 64 output tile; each wave owns a
// 32 x 32 quarter as 2 x 2 MFMA 16x16 blocks; k advances 16 at a time through
// LDS, 4 per MFMA. MFMA 16x16x4 lane mapping: lane l supplies A(l%16, l/16)
// and B(l/16, l%16); its accumulator register r holds C(row, l%16) with
// row = 4*(l/16) + r for FP32 and row = l/16 + 4*r for FP64 (the FP64
// instruction interleaves its output rows).
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace nce {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <class T>
struct Mfma;
template <>
struct Mfma<double> {
    typedef v4d acc_t;
    static __device__ __forceinline__ int row(int lk, int r) { return lk + 4 * r; }
    static __device__ __forceinline__ acc_t step(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mfma<float> {
    typedef v4f acc_t;
    static __device__ __forceinline__ int row(int lk, int r) { return 4 * lk + r; }
    static __device__ __forceinline__ acc_t step(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

template <class T, class TO>
__global__ __launch_bounds__(256) void k_gemm_mfma(int m, int n, int k, const T* __restrict__ A, int64_t sai,
                                                   int64_t sak, const T* __restrict__ B, int64_t sbk, int64_t sbj,
                                                   TO* __restrict__ C, int64_t ldc, T alpha, int accumulate,
                                                   const double* __restrict__ D, int64_t ldd) {
    __shared__ T As[16][64 + 1];  // [k][row]
    __shared__ T Bs[16][64 + 1];  // [k][col]
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
    const int wr = (wave / 2) * 32, wc = (wave % 2) * 32;
    typedef typename Mfma<T>::acc_t acc_t;
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[a][b][r] = T(0);
    const int lr = lane % 16, lk = lane / 16;
    for (int k0 = 0; k0 < k; k0 += 16) {
        // consecutive threads walk the operand's contiguous index (k when the
        // k stride is 1, the row or column otherwise) so that loads coalesce
        const bool a_k = sak == 1, b_k = sbk == 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int idx = threadIdx.x + 256 * r;  // 0..1023
            const int ra = a_k ? idx / 16 : idx % 64, ka = a_k ? idx % 16 : idx / 64;
            const int cb = b_k ? idx / 16 : idx % 64, kb = b_k ? idx % 16 : idx / 64;
            const int gi = i0 + ra, gka = k0 + ka, gj = j0 + cb, gkb = k0 + kb;
            As[ka][ra] = (gi < m && gka < k) ? A[gi * sai + gka * sak] : T(0);
            Bs[kb][cb] = (gj < n && gkb < k) ? B[gkb * sbk + gj * sbj] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            T av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kk + lk][wr + a * 16 + lr];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kk + lk][wc + b * 16 + lr];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = Mfma<T>::step(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gi = i0 + wr + a * 16 + Mfma<T>::row(lk, r);
                const int gj = j0 + wc + b * 16 + lr;
                if (gi < m && gj < n) {
                    T v = alpha * acc[a][b][r];
                    TO* c = C + gi * ldc + gj;
                    if (D)
                        *c = (TO)((double)v + D[gi * ldd + gj]);
                    else if (accumulate)
                        *c = (TO)((T)*c + v);
                    else
                        *c = (TO)v;
                }
            }
}

}  // namespace

template <class T>
hipError_t gemm_strided(hipStream_t s, int m, int n, int k, const T* A, int64_t sai, int64_t sak, const T* B,
                        int64_t sbk, int64_t sbj, T* C, int64_t ldc, T alpha, int accumulate) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((n + 63) / 64, (m + 63) / 64);
    hipLaunchKernelGGL((k_gemm_mfma<T, T>), grid, dim3(256), 0, s, m, n, k, A, sai, sak, B, sbk, sbj, C, ldc, alpha,
                       accumulate, (const double*)nullptr, (int64_t)0);
    return hipGetLastError();
}
template hipError_t gemm_strided<double>(hipStream_t, int, int, int, const double*, int64_t, int64_t, const double*,
                                         int64_t, int64_t, double*, int64_t, double, int);
template hipError_t gemm_strided<float>(hipStream_t, int, int, int, const float*, int64_t, int64_t, const float*,
                                        int64_t, int64_t, float*, int64_t, float, int);

template <class T>
hipError_t gemm_nt(hipStream_t s, int m, int n, int k, const T* A, int lda, const T* B, int ldb, T* C, int ldc,
                   const double* D, int ldd) {
    if (m <= 0 || n <= 0) return hipSuccess;
    dim3 grid((n + 63) / 64, (m + 63) / 64);
    hipLaunchKernelGGL((k_gemm_mfma<T, T>), grid, dim3(256), 0, s, m, n, k, A, (int64_t)lda, (int64_t)1, B,
                       (int64_t)1, (int64_t)ldb, C, (int64_t)ldc, T(1), 0, D, (int64_t)ldd);
    return hipGetLastError();
}
template hipError_t gemm_nt<double>(hipStream_t, int, int, int, const double*, int, const double*, int, double*, int,
                                    const double*, int);
template hipError_t gemm_nt<float>(hipStream_t, int, int, int, const float*, int, const float*, int, float*, int,
                                   const double*, int);

template <class T>
hipError_t p_apply(hipStream_t s, int N, int K, int Kstar, const T* U, const T* P, const double* x, double* y) {
    dim3 grid((K + 63) / 64, (N + 63) / 64);
    hipLaunchKernelGGL((k_gemm_mfma<T, double>), grid, dim3(256), 0, s, N, K, Kstar, U, (int64_t)Kstar, (int64_t)1,
                       P, (int64_t)1, (int64_t)Kstar, y, (int64_t)K, T(1), 0, x, (int64_t)K);
    return hipGetLastError();
}
template hipError_t p_apply<double>(hipStream_t, int, int, int, const double*, const double*, const double*, double*);
template hipError_t p_apply<float>(hipStream_t, int, int, int, const float*, const float*, const double*, double*);

}  // namespace nce
