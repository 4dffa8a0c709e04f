// Host part of the coarse-space deflation (see deflate.hpp): the orthonormal
// basis of the polynomials of degree <= 3 on the patch centres.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace nce {

constexpr int kDeflHost = 16;
// Reductions run over this many fixed index ranges whose partial sums are
// added in range order, so the basis (and every solve that uses it) is the
// same bit for bit whatever the thread count and scheduling.
constexpr int kChunks = 64;
// inner loops run in parallel only for configurations at least this large
// (below it a parallel region costs more than the loop)
constexpr int kParMin = 16384;

namespace {

inline void chunk_range(int N, int c, int& i0, int& i1) {
    i0 = (int)((int64_t)N * c / kChunks);
    i1 = (int)((int64_t)N * (c + 1) / kChunks);
}

// sum over i of a[i] b[i], deterministic
double dot_det(const double* a, const double* b, int N) {
    double part[kChunks];
#pragma omp parallel for schedule(static) if (N >= kParMin)
    for (int c = 0; c < kChunks; ++c) {
        int i0, i1;
        chunk_range(N, c, i0, i1);
        double s = 0.0;
        for (int i = i0; i < i1; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < kChunks; ++c) s += part[c];
    return s;
}

}  // namespace

// The 16 harmonic polynomials of degree <= 3 (a basis of that space on the
// sphere), orthonormalized over the centres by modified Gram-Schmidt, twice.
int deflation_basis(const std::vector<double>& frames, int N, std::vector<double>& Z) {
    std::vector<double> C((size_t)kDeflHost * N);  // column-major candidates
#pragma omp parallel for schedule(static) if (N >= kParMin)
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
        const double n0 = dot_det(v, v, N);
        for (int pass = 0; pass < 2; ++pass)
            for (int u = 0; u < k; ++u) {
                const double* q = &C[(size_t)u * N];
                const double d = dot_det(q, v, N);
#pragma omp parallel for schedule(static) if (N >= kParMin)
                for (int i = 0; i < N; ++i) v[i] -= d * q[i];
            }
        const double n1 = dot_det(v, v, N);
        if (n1 > 1e-16 * n0 && n1 > 0.0) {
            const double s = 1.0 / std::sqrt(n1);
            double* dst = &C[(size_t)k * N];
            for (int i = 0; i < N; ++i) dst[i] = v[i] * s;
            ++k;
        }
    }
    Z.assign((size_t)N * kDeflHost, 0.0);
#pragma omp parallel for schedule(static) if (N >= kParMin)
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
    std::vector<double> part((size_t)kChunks * k * k, 0.0);
#pragma omp parallel for schedule(static) if (N >= kParMin)
    for (int c = 0; c < kChunks; ++c) {
        int i0, i1;
        chunk_range(N, c, i0, i1);
        double* loc = &part[(size_t)c * k * k];
        for (int i = i0; i < i1; ++i)
            for (int a = 0; a < k; ++a) {
                const double za = Z[(size_t)i * kDeflHost + a];
                for (int b = 0; b < k; ++b) loc[(size_t)a * k + b] += za * S[(size_t)i * kDeflHost + b];
            }
    }
    for (int c = 0; c < kChunks; ++c)
        for (size_t e = 0; e < G.size(); ++e) G[e] += part[(size_t)c * k * k + e];
}

// M = T^{-1} - I (kDeflHost x kDeflHost, zero beyond k) for the k x k
// coarse matrix T (row-major), by Gauss-Jordan elimination with partial
// pivoting. Returns false if T is singular.
bool deflation_invert(std::vector<double> T, int k, std::vector<double>& M) {
    M.assign((size_t)kDeflHost * kDeflHost, 0.0);
    std::vector<double> inv((size_t)k * k, 0.0);
    for (int a = 0; a < k; ++a) inv[(size_t)a * k + a] = 1.0;
    for (int col = 0; col < k; ++col) {
        int piv = col;
        for (int r = col + 1; r < k; ++r)
            if (std::fabs(T[(size_t)r * k + col]) > std::fabs(T[(size_t)piv * k + col])) piv = r;
        if (!(std::fabs(T[(size_t)piv * k + col]) > 0.0)) return false;
        for (int c = 0; c < k; ++c) {
            std::swap(T[(size_t)col * k + c], T[(size_t)piv * k + c]);
            std::swap(inv[(size_t)col * k + c], inv[(size_t)piv * k + c]);
        }
        const double d = T[(size_t)col * k + col];
        for (int c = 0; c < k; ++c) {
            T[(size_t)col * k + c] /= d;
            inv[(size_t)col * k + c] /= d;
        }
        for (int r = 0; r < k; ++r)
            if (r != col) {
                const double f = T[(size_t)r * k + col];
                for (int c = 0; c < k; ++c) {
                    T[(size_t)r * k + c] -= f * T[(size_t)col * k + c];
                    inv[(size_t)r * k + c] -= f * inv[(size_t)col * k + c];
                }
            }
    }
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) M[(size_t)a * kDeflHost + b] = inv[(size_t)a * k + b] - (a == b ? 1.0 : 0.0);
    return true;
}

// T = I + chi0 Z^T S on the k independent columns (Z^T Z = I), k x k
void deflation_coarse_matrix(const std::vector<double>& Z, const std::vector<double>& S, int N, int k, double chi0,
                             std::vector<double>& T) {
    deflation_gram(Z, S, N, k, T);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b) T[(size_t)a * k + b] = (a == b ? 1.0 : 0.0) + chi0 * T[(size_t)a * k + b];
}

// Bases of many configurations at once, in parallel over configurations:
// configuration c has N[c] patches with frames fr[c] (9 per patch) and its
// rows at Zall + 16 off[c]; those with N[c] < nmin are left zero (k[c] = 0).
void deflation_bases(int ncfg, const double* const* fr, const int* N, const int64_t* off, int nmin, double* Zall,
                     int* k) {
#pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < ncfg; ++c) {
        k[c] = 0;
        if (N[c] < nmin) continue;
        const std::vector<double> frames(fr[c], fr[c] + (size_t)9 * N[c]);
        std::vector<double> Z;
        k[c] = deflation_basis(frames, N[c], Z);
        std::copy(Z.begin(), Z.end(), Zall + (size_t)off[c] * kDeflHost);
    }
}

// M_c = T_c^{-1} - I of many configurations (Zall, Sall as for
// deflation_bases; Mall: ncfg x 16 x 16, zero where k[c] = 0 or where T_c is
// singular, which leaves that configuration undeflated). Returns how many
// configurations had a singular T.
int deflation_inverses(int ncfg, const int* N, const int64_t* off, const int* k, const double* chi0,
                       const double* Zall, const double* Sall, double* Mall) {
    int bad = 0;
#pragma omp parallel for schedule(dynamic)
    for (int c = 0; c < ncfg; ++c) {
        double* Mc = Mall + (size_t)c * kDeflHost * kDeflHost;
        std::fill(Mc, Mc + kDeflHost * kDeflHost, 0.0);
        if (k[c] == 0) continue;
        const size_t a0 = (size_t)off[c] * kDeflHost, a1 = a0 + (size_t)N[c] * kDeflHost;
        const std::vector<double> Z(Zall + a0, Zall + a1), S(Sall + a0, Sall + a1);
        std::vector<double> T, M;
        deflation_coarse_matrix(Z, S, N[c], k[c], chi0[c], T);
        if (!deflation_invert(T, k[c], M)) {
#pragma omp atomic
            ++bad;
            continue;
        }
        std::copy(M.begin(), M.end(), Mc);
    }
    return bad;
}

}  // namespace nce
