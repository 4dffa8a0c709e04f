// Host computation of the warm-start network's per-patch features (see mlp.hpp).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <utility>
#include <vector>

namespace nce {

constexpr int kFeatureDimHost = 56;

static inline double geod(const double* a, const double* b) {
    double c0 = a[1] * b[2] - a[2] * b[1], c1 = a[2] * b[0] - a[0] * b[2], c2 = a[0] * b[1] - a[1] * b[0];
    return std::atan2(std::sqrt(c0 * c0 + c1 * c1 + c2 * c2), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

// Per patch i: the 16 nearest other patches (by geodesic distance between
// centres; equivalently by chord, which is monotone in it) in the patch's
// frame, the patch counts within 8, 16, 32 and 64 eps relative to a uniform
// layout, the problem, the area fraction and the coarse amplitude. Neighbours
// come from a uniform grid of cubic cells over [-1, 1]^3 (cell side = chord of
// 64 eps), searched in growing cubes until the 16th neighbour and the largest
// radius lie inside the searched ball.
void patch_features_geometry(const std::vector<double>& frames, int64_t N, double eps, int problem,
                             std::vector<float>& out) {
    out.assign((size_t)N * kFeatureDimHost, 0.0f);
    const double radii[4] = {8 * eps, 16 * eps, 32 * eps, 64 * eps};
    double chord2[4];
    for (int q = 0; q < 4; ++q) {
        const double R = std::min(radii[q], M_PI);
        chord2[q] = 4.0 * std::sin(0.5 * R) * std::sin(0.5 * R);
    }
    const double area = N * std::sin(0.5 * eps) * std::sin(0.5 * eps);  // patch area fraction (Section 10)
    const double h = std::max(2.0 * std::sin(std::min(32.0 * eps, 1.5)), 1e-3);  // chord of 64 eps (cell size)
    const int64_t nc = (int64_t)std::ceil(2.0 / h) + 2;
    auto cell = [&](double v) { return std::min<int64_t>(nc - 1, std::max<int64_t>(0, (int64_t)std::floor((v + 1.0) / h))); };
    // cells as CSR over a dense nc^3 index (counting sort of the patches)
    std::vector<int64_t> cid((size_t)N);
    std::vector<int> start((size_t)(nc * nc * nc + 1), 0), order((size_t)N);
    for (int64_t i = 0; i < N; ++i) {
        const double* c = &frames[(size_t)i * 9];
        cid[i] = (cell(c[0]) * nc + cell(c[1])) * nc + cell(c[2]);
        start[cid[i] + 1]++;
    }
    for (size_t k = 1; k < start.size(); ++k) start[k] += start[k - 1];
    {
        std::vector<int> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < N; ++i) order[fill[cid[i]]++] = (int)i;
    }
    // centres in cell order, so that a cell's candidates are read contiguously
    std::vector<double> cs((size_t)N * 3);
    for (int64_t s = 0; s < N; ++s)
        for (int d = 0; d < 3; ++d) cs[(size_t)s * 3 + d] = frames[(size_t)order[s] * 9 + d];
#pragma omp parallel
    {
        std::vector<std::pair<double, int>> cand;
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < N; ++i) {
            const double* f = &frames[(size_t)i * 9];
            const int64_t cx = cell(f[0]), cy = cell(f[1]), cz = cell(f[2]);
            int reach = 1;
            int nn = 0;
            while (true) {
                cand.clear();
                for (int64_t x = std::max<int64_t>(0, cx - reach); x <= std::min(nc - 1, cx + reach); ++x)
                    for (int64_t y = std::max<int64_t>(0, cy - reach); y <= std::min(nc - 1, cy + reach); ++y)
                        for (int64_t z = std::max<int64_t>(0, cz - reach); z <= std::min(nc - 1, cz + reach); ++z) {
                            const int64_t k = (x * nc + y) * nc + z;
                            for (int s = start[k]; s < start[k + 1]; ++s) {
                                const int j = order[s];
                                if (j == i) continue;
                                const double* g = &cs[(size_t)s * 3];
                                const double d0 = g[0] - f[0], d1 = g[1] - f[1], d2 = g[2] - f[2];
                                cand.push_back({d0 * d0 + d1 * d1 + d2 * d2, j});
                            }
                        }
                // every patch within chord reach*h of the centre has been seen
                const double safe = std::min(2.0, reach * h);
                const double safe2 = safe * safe;
                const bool whole = reach * h > 2.5;
                nn = std::min<int>(16, (int)cand.size());
                std::partial_sort(cand.begin(), cand.begin() + nn, cand.end());
                if (whole || (nn == 16 && cand[15].first <= safe2 && chord2[3] <= safe2)) break;
                reach++;
            }
            float* o = &out[(size_t)i * kFeatureDimHost];
            for (int k = 0; k < nn; ++k) {
                const double* g = &frames[(size_t)cand[k].second * 9];
                const double d[3] = {g[0] - f[0], g[1] - f[1], g[2] - f[2]};
                const double u = (d[0] * f[3] + d[1] * f[4] + d[2] * f[5]) / eps;
                const double v = (d[0] * f[6] + d[1] * f[7] + d[2] * f[8]) / eps;
                const double r = geod(f, g) / eps;
                o[3 * k] = (float)(u / 16.0);
                o[3 * k + 1] = (float)(v / 16.0);
                o[3 * k + 2] = (float)(4.0 / r);
            }
            o[48] = (float)problem;
            o[49] = (float)(10.0 * area);
            int cnt[4] = {0, 0, 0, 0};
            for (const auto& pr : cand)
                for (int q = 0; q < 4; ++q) cnt[q] += pr.first <= chord2[q];
            for (int q = 0; q < 4; ++q) {
                const double R = std::min(radii[q], M_PI);
                const double expect = std::max((N - 1) * 0.5 * (1.0 - std::cos(R)), 1e-12);
                o[50 + q] = (float)(cnt[q] / expect);
            }
        }
    }
}

void patch_features_amplitudes(const std::vector<double>& a, int64_t N, std::vector<float>& out) {
    double amean = 0.0;
    for (int64_t i = 0; i < N; ++i) amean += a[i];
    amean /= (double)N;
    for (int64_t i = 0; i < N; ++i) {
        float* o = &out[(size_t)i * kFeatureDimHost];
        o[54] = (float)(10.0 * (a[i] / amean - 1.0));
        o[55] = (float)amean;
    }
}

void patch_features(const std::vector<double>& frames, int64_t N, double eps, int problem,
                    const std::vector<double>& a, std::vector<float>& out) {
    patch_features_geometry(frames, N, eps, problem, out);
    patch_features_amplitudes(a, N, out);
}

}  // namespace nce
