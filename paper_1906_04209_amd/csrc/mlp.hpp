// Warm-start network (FP32 MLP) held on the device; see mlp.hip.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace nce {

struct Mlp {
    int n_in, width, hidden, n_out;
    int64_t nparam = 0;
    std::vector<int> lin, lout;
    std::vector<int64_t> woff, boff;
    float* theta = nullptr;
    float* grad = nullptr;
    float* mom = nullptr;
    float* vel = nullptr;
    double* partial = nullptr;
    double* lossd = nullptr;   // device: sum of squared errors of the last loss_grad
    int64_t step = 0;
    // activations of the last forward pass (per layer: pre-activation Z, output H)
    int64_t cap = 0;
    std::vector<float*> Z, H;
    float* G0 = nullptr;
    float* G1 = nullptr;

    Mlp(int n_in, int width, int hidden, int n_out, uint64_t seed);
    ~Mlp();
    Mlp(const Mlp&) = delete;
    Mlp& operator=(const Mlp&) = delete;
    void ensure(int64_t B);
    void release_ws();
    // returns the device output (B x n_out), valid until the next call
    const float* forward(hipStream_t s, const float* x, int64_t B);
    // widest hidden layer (0 without hidden layers)
    int64_t widest_hidden() const;
    // the same forward pass with no allocation: the hidden activations go to
    // the caller's device workspace ws (ws_floats floats, two row-chunks of the
    // widest hidden layer), rows in chunks that fit it, the output straight to
    // y (B x n_out); nothing else is written
    void forward_ws(hipStream_t s, const float* x, int64_t B, float* y, float* ws, int64_t ws_floats);
    // forward + MSE gradient into `grad`; squared-error sum into lossd
    void loss_grad(hipStream_t s, const float* x, const float* t, int64_t B);
    void adam_step(hipStream_t s, float lr);
};

// Per-patch input features of the warm-start network (host): the 16 nearest
// neighbours' positions in the patch frame (scaled by 1/eps) and inverse
// distances, the problem flag, the area fraction, the neighbour density
// relative to uniform within 8, 16, 32 and 64 eps, and the patch's coarse
// amplitude relative to the layout mean with that mean itself.
// frames: N x 9 (c, e1, e2); a: the N coarse amplitudes.
constexpr int kFeatureDim = 56;
void patch_features(const std::vector<double>& frames, int64_t N, double eps, int problem,
                    const std::vector<double>& a, std::vector<float>& out);
// The same in two parts: everything but the amplitude features (sizes out),
// then the two amplitude features, so that the first part can run on the host
// while the coarse solve runs on the device.
void patch_features_geometry(const std::vector<double>& frames, int64_t N, double eps, int problem,
                             std::vector<float>& out);
void patch_features_amplitudes(const std::vector<double>& a, int64_t N, std::vector<float>& out);

}  // namespace nce
