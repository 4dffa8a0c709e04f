// Host part of the coarse-space deflation (see deflate.hpp): the orthonormal
// basis of the polynomials of degree <= 3 on the patch centres.
#include <cmath>
#include <cstdint>
#include <vector>

namespace nce {

constexpr int kDeflHost = 16;

// The 16 harmonic polynomials of degree <= 3 (a basis of that space on the
// sphere), orthonormalized over the centres by modified Gram-Schmidt, twice.
int deflation_basis(const std::vector<double>& frames, int N, std::vector<double>& Z) {
    std::vector<double> C((size_t)kDeflHost * N);  // column-major candidates
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i) {
        const double x = frames[(size_t)i * 9], y = frames[(size_t)i * 9 + 1], z = frames[(size_t)i * 9 + 2];
        const double r2 = x * x + y * y;
        const double v[kDeflHost] = {1.0,
                                     x, y, z,
                                     x * y, y * z, z * x, x * x - y * y, 2 * z * z - r2,
                                     x * (x * x - 3 * y * y), y * (3 * x * x - y * y), z * (x * x - y * y), x * y * z,
                                     x * (4 * z * z - r2), y * (4 * z * z - r2), z * (2 * z * z - 3 * r2)};
        for (int c = 0; c < kDeflHost; ++c) C[(size_t)c * N + i] = v[c];
    }
    int k = 0;
    for (int c = 0; c < kDeflHost; ++c) {
        double* v = &C[(size_t)c * N];
        double n0 = 0.0;
#pragma omp parallel for reduction(+ : n0) schedule(static)
        for (int i = 0; i < N; ++i) n0 += v[i] * v[i];
        for (int pass = 0; pass < 2; ++pass)
            for (int u = 0; u < k; ++u) {
                const double* q = &C[(size_t)u * N];
                double d = 0.0;
#pragma omp parallel for reduction(+ : d) schedule(static)
                for (int i = 0; i < N; ++i) d += q[i] * v[i];
#pragma omp parallel for schedule(static)
                for (int i = 0; i < N; ++i) v[i] -= d * q[i];
            }
        double n1 = 0.0;
#pragma omp parallel for reduction(+ : n1) schedule(static)
        for (int i = 0; i < N; ++i) n1 += v[i] * v[i];
        if (n1 > 1e-16 * n0 && n1 > 0.0) {
            const double s = 1.0 / std::sqrt(n1);
            double* dst = &C[(size_t)k * N];
            for (int i = 0; i < N; ++i) dst[i] = v[i] * s;
            ++k;
        }
    }
    Z.assign((size_t)N * kDeflHost, 0.0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < N; ++i)
        for (int c = 0; c < k; ++c) Z[(size_t)i * kDeflHost + c] = C[(size_t)c * N + i];
    return k;
}

}  // namespace nce

namespace nce {

// G = Z^T S on the first k columns (Z, S: N x 16 row-major); k x k row-major.
void deflation_gram(const std::vector<double>& Z, const std::vector<double>& S, int N, int k,
                    std::vector<double>& G) {
    G.assign((size_t)k * k, 0.0);
#pragma omp parallel
    {
        std::vector<double> loc((size_t)k * k, 0.0);
#pragma omp for schedule(static)
        for (int i = 0; i < N; ++i)
            for (int a = 0; a < k; ++a) {
                const double za = Z[(size_t)i * kDeflHost + a];
                for (int b = 0; b < k; ++b) loc[(size_t)a * k + b] += za * S[(size_t)i * kDeflHost + b];
            }
#pragma omp critical
        for (size_t e = 0; e < loc.size(); ++e) G[e] += loc[e];
    }
}

}  // namespace nce
