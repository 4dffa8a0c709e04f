// Warm-start network on the GPU: an FP32 multilayer perceptron (SiLU hidden
// layers, linear output) with its forward pass, mean-squared-error gradient by
// backpropagation and Adam updates, all as device kernels around the MFMA GEMM.
// Parameter layout: per layer W (row-major, n_out_l x n_in_l) then b.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <random>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "mlp.hpp"

namespace nce {

namespace {

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__global__ void k_bias_act(int64_t B, int n, const float* __restrict__ bias, float* __restrict__ Z,
                           float* __restrict__ H, int act) {
    const int64_t total = B * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float z = Z[e] + bias[e % n];
        Z[e] = z;
        H[e] = act ? silu(z) : z;
    }
}

// the same, in place (X = act(X + b)): the allocation-free forward pass
__global__ void k_bias_act_inplace(int64_t B, int n, const float* __restrict__ bias, float* __restrict__ X, int act) {
    const int64_t total = B * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float z = X[e] + bias[e % n];
        X[e] = act ? silu(z) : z;
    }
}

__global__ void k_silu_back(int64_t total, const float* __restrict__ Z, float* __restrict__ G) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        G[e] *= dsilu(Z[e]);
}

// G = scale (Y - T); per-block partial sums of (Y - T)^2 (FP64)
__global__ __launch_bounds__(256) void k_mse(int64_t total, const float* __restrict__ Y, const float* __restrict__ T,
                                             float scale, float* __restrict__ G, double* __restrict__ partial) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const float d = Y[e] - T[e];
        G[e] = scale * d;
        acc += (double)d * d;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// out[j] = sum_i G[i][j] (one block per column chunk of 64; threads stride rows)
__global__ __launch_bounds__(256) void k_colsum(int64_t B, int n, const float* __restrict__ G, float* __restrict__ out) {
    __shared__ float red[4][64];
    const int j = blockIdx.x * 64 + threadIdx.x % 64;
    const int rw = threadIdx.x / 64;
    float acc = 0.0f;
    if (j < n)
        for (int64_t i = rw; i < B; i += 4) acc += G[i * n + j];
    red[rw][threadIdx.x % 64] = acc;
    __syncthreads();
    if (rw == 0 && j < n) out[j] = red[0][threadIdx.x] + red[1][threadIdx.x] + red[2][threadIdx.x] + red[3][threadIdx.x];
}

__global__ void k_adam(int64_t n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const float gg = g[e];
        const float mm = b1 * m[e] + (1.0f - b1) * gg;
        const float vv = b2 * v[e] + (1.0f - b2) * gg * gg;
        m[e] = mm;
        v[e] = vv;
        th[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
    }
}

__global__ void k_sum_partials_f(int nb, const double* __restrict__ partial, double* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += partial[b];
        out[0] = s;
    }
}

dim3 ew(int64_t n) {
    int64_t b = (n + 255) / 256;
    return dim3((unsigned)(b < 4096 ? (b < 1 ? 1 : b) : 4096));
}

void chk(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

Mlp::Mlp(int n_in_, int width_, int hidden_, int n_out_, uint64_t seed) : n_in(n_in_), width(width_), hidden(hidden_),
                                                                          n_out(n_out_) {
    std::vector<int> dims{n_in};
    for (int h = 0; h < hidden; ++h) dims.push_back(width);
    dims.push_back(n_out);
    nparam = 0;
    for (size_t l = 0; l + 1 < dims.size(); ++l) {
        lin.push_back(dims[l]);
        lout.push_back(dims[l + 1]);
        woff.push_back(nparam);
        nparam += (int64_t)dims[l] * dims[l + 1];
        boff.push_back(nparam);
        nparam += dims[l + 1];
    }
    std::vector<float> th(nparam, 0.0f);
    std::mt19937_64 g(seed);
    for (size_t l = 0; l < lin.size(); ++l) {
        std::normal_distribution<float> nd(0.0f, std::sqrt(2.0f / lin[l]));
        for (int64_t q = 0; q < (int64_t)lin[l] * lout[l]; ++q) th[woff[l] + q] = nd(g);
    }
    chk(hipMalloc((void**)&theta, nparam * sizeof(float)), "hipMalloc");
    chk(hipMalloc((void**)&grad, nparam * sizeof(float)), "hipMalloc");
    chk(hipMalloc((void**)&mom, nparam * sizeof(float)), "hipMalloc");
    chk(hipMalloc((void**)&vel, nparam * sizeof(float)), "hipMalloc");
    chk(hipMalloc((void**)&partial, 4096 * sizeof(double)), "hipMalloc");
    chk(hipMalloc((void**)&lossd, 8 * sizeof(double)), "hipMalloc");
    chk(hipMemcpy(theta, th.data(), nparam * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy");
    chk(hipMemset(mom, 0, nparam * sizeof(float)), "hipMemset");
    chk(hipMemset(vel, 0, nparam * sizeof(float)), "hipMemset");
}

Mlp::~Mlp() {
    release_ws();
    for (void* p : {(void*)theta, (void*)grad, (void*)mom, (void*)vel, (void*)partial, (void*)lossd})
        if (p) (void)hipFree(p);
}

void Mlp::release_ws() {
    for (float* p : Z) (void)hipFree(p);
    for (float* p : H) (void)hipFree(p);
    if (G0) (void)hipFree(G0);
    if (G1) (void)hipFree(G1);
    Z.clear();
    H.clear();
    G0 = G1 = nullptr;
    cap = 0;
}

void Mlp::ensure(int64_t B) {
    if (B <= cap) return;
    release_ws();
    int mx = n_in;
    for (size_t l = 0; l < lout.size(); ++l) {
        float *z = nullptr, *h = nullptr;
        chk(hipMalloc((void**)&z, (size_t)B * lout[l] * sizeof(float)), "hipMalloc");
        chk(hipMalloc((void**)&h, (size_t)B * lout[l] * sizeof(float)), "hipMalloc");
        Z.push_back(z);
        H.push_back(h);
        mx = std::max(mx, lout[l]);
    }
    chk(hipMalloc((void**)&G0, (size_t)B * mx * sizeof(float)), "hipMalloc");
    chk(hipMalloc((void**)&G1, (size_t)B * mx * sizeof(float)), "hipMalloc");
    cap = B;
}

const float* Mlp::forward(hipStream_t s, const float* x, int64_t B) {
    ensure(B);
    const float* in = x;
    for (size_t l = 0; l < lout.size(); ++l) {
        // Z = in W^T (A(i,k) = in[i*n_in_l + k], B(k,j) = W[j*n_in_l + k])
        chk(gemm_strided<float>(s, (int)B, lout[l], lin[l], in, lin[l], 1, theta + woff[l], 1, lin[l], Z[l], lout[l],
                                1.0f, 0),
            "gemm");
        hipLaunchKernelGGL(k_bias_act, ew(B * lout[l]), dim3(256), 0, s, B, lout[l], theta + boff[l], Z[l], H[l],
                           (int)(l + 1 < lout.size()));
        chk(hipGetLastError(), "bias_act");
        in = H[l];
    }
    return H.back();
}

int64_t Mlp::widest_hidden() const {
    int64_t w = 0;
    for (size_t l = 0; l + 1 < lout.size(); ++l) w = std::max<int64_t>(w, lout[l]);
    return w;
}

void Mlp::forward_ws(hipStream_t s, const float* x, int64_t B, float* y, float* ws, int64_t ws_floats) {
    const size_t L = lout.size();
    const int64_t wmax = widest_hidden();
    // rows per chunk: two activation buffers of rows x wmax floats must fit
    const int64_t rows = std::min<int64_t>(B, ws_floats / (2 * std::max<int64_t>(wmax, 1)));
    if (rows < 1) throw std::runtime_error("workspace holds less than one row of activations");
    float* buf[2] = {ws, ws + rows * wmax};
    for (int64_t r0 = 0; r0 < B; r0 += rows) {
        const int64_t nb = std::min(rows, B - r0);
        const float* in = x + r0 * n_in;
        for (size_t l = 0; l < L; ++l) {
            float* out = l + 1 == L ? y + r0 * n_out : buf[l % 2];
            chk(gemm_strided<float>(s, (int)nb, lout[l], lin[l], in, lin[l], 1, theta + woff[l], 1, lin[l], out,
                                    lout[l], 1.0f, 0),
                "gemm");
            hipLaunchKernelGGL(k_bias_act_inplace, ew(nb * lout[l]), dim3(256), 0, s, nb, lout[l], theta + boff[l],
                               out, (int)(l + 1 < L));
            chk(hipGetLastError(), "bias_act");
            in = out;
        }
    }
}

void Mlp::loss_grad(hipStream_t s, const float* x, const float* t, int64_t B) {
    forward(s, x, B);
    const size_t L = lout.size();
    const int64_t ny = B * n_out;
    const int nb = (int)ew(ny).x;
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, ny, H.back(), t, 2.0f / (float)ny, G0, partial);
    hipLaunchKernelGGL(k_sum_partials_f, dim3(1), dim3(64), 0, s, nb, partial, lossd);
    chk(hipGetLastError(), "mse");
    float* G = G0;
    float* Gn = G1;
    for (int l = (int)L - 1; l >= 0; --l) {
        if (l < (int)L - 1) {
            hipLaunchKernelGGL(k_silu_back, ew(B * lout[l]), dim3(256), 0, s, B * lout[l], Z[l], G);
            chk(hipGetLastError(), "silu_back");
        }
        const float* in = l == 0 ? x : H[l - 1];
        // dW = G^T in: A(i,k) = G[k*out + i], B(k,j) = in[k*n_in_l + j]
        chk(gemm_strided<float>(s, lout[l], lin[l], (int)B, G, 1, lout[l], in, lin[l], 1, grad + woff[l], lin[l], 1.0f,
                                0),
            "gemm dW");
        hipLaunchKernelGGL(k_colsum, dim3((lout[l] + 63) / 64), dim3(256), 0, s, B, lout[l], G, grad + boff[l]);
        chk(hipGetLastError(), "colsum");
        if (l > 0) {
            // G_prev = G W: A(i,k) = G[i*out + k], B(k,j) = W[k*n_in_l + j]
            chk(gemm_strided<float>(s, (int)B, lin[l], lout[l], G, lout[l], 1, theta + woff[l], lin[l], 1, Gn,
                                    lin[l], 1.0f, 0),
                "gemm dX");
            std::swap(G, Gn);
        }
    }
}

void Mlp::adam_step(hipStream_t s, float lr) {
    ++step;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(k_adam, ew(nparam), dim3(256), 0, s, nparam, theta, grad, mom, vel, lr, b1, b2, 1e-8f, c1, c2);
    chk(hipGetLastError(), "adam");
}

}  // namespace nce
