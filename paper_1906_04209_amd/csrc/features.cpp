// Host computation of the warm-start network's per-patch features (see mlp.hpp).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_map>
#include <vector>

namespace nce {

constexpr int kFeatureDimHost = 56;

static inline double geod(const double* a, const double* b) {
    double c0 = a[1] * b[2] - a[2] * b[1], c1 = a[2] * b[0] - a[0] * b[2], c2 = a[0] * b[1] - a[1] * b[0];
    return std::atan2(std::sqrt(c0 * c0 + c1 * c1 + c2 * c2), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

void patch_features(const std::vector<double>& frames, int64_t N, double eps, int problem,
                    const std::vector<double>& a, std::vector<float>& out) {
    out.assign((size_t)N * kFeatureDimHost, 0.0f);
    double amean = 0.0;
    for (int64_t i = 0; i < N; ++i) amean += a[i];
    amean /= (double)N;
    const double radii[4] = {8 * eps, 16 * eps, 32 * eps, 64 * eps};
    const double area = N * std::sin(0.5 * eps) * std::sin(0.5 * eps);  // patch area fraction (Section 10)
    const double h = std::max(2.0 * std::sin(std::min(32.0 * eps, 1.5)), 1e-3);  // chord of 64 eps (cell size)
    const int64_t nc = (int64_t)std::ceil(2.0 / h) + 2;
    auto cell = [&](double v) { return (int64_t)std::floor((v + 1.0) / h); };
    std::unordered_map<int64_t, std::vector<int>> grid;
    grid.reserve((size_t)N * 2);
    for (int64_t i = 0; i < N; ++i) {
        const double* c = &frames[(size_t)i * 9];
        grid[(cell(c[0]) * nc + cell(c[1])) * nc + cell(c[2])].push_back((int)i);
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < N; ++i) {
        const double* f = &frames[(size_t)i * 9];
        const int64_t cx = cell(f[0]), cy = cell(f[1]), cz = cell(f[2]);
        std::vector<std::pair<double, int>> cand;
        int reach = 1;
        while (true) {
            cand.clear();
            for (int64_t dx = -reach; dx <= reach; ++dx)
                for (int64_t dy = -reach; dy <= reach; ++dy)
                    for (int64_t dz = -reach; dz <= reach; ++dz) {
                        auto it = grid.find(((cx + dx) * nc + (cy + dy)) * nc + (cz + dz));
                        if (it == grid.end()) continue;
                        for (int j : it->second)
                            if (j != i) cand.push_back({geod(f, &frames[(size_t)j * 9]), j});
                    }
            // enough neighbours found inside the searched ball (or the whole sphere searched)
            const double safe = 2.0 * std::asin(std::min(1.0, 0.5 * reach * h));
            std::sort(cand.begin(), cand.end());
            const bool whole = reach * h > 2.5;
            if (whole || ((int)cand.size() >= 16 && cand[15].first <= safe && radii[3] <= safe)) break;
            reach++;
        }
        float* o = &out[(size_t)i * kFeatureDimHost];
        for (int k = 0; k < 16 && k < (int)cand.size(); ++k) {
            const double* g = &frames[(size_t)cand[k].second * 9];
            const double d[3] = {g[0] - f[0], g[1] - f[1], g[2] - f[2]};
            const double u = (d[0] * f[3] + d[1] * f[4] + d[2] * f[5]) / eps;
            const double v = (d[0] * f[6] + d[1] * f[7] + d[2] * f[8]) / eps;
            const double r = cand[k].first / eps;
            o[3 * k] = (float)(u / 16.0);
            o[3 * k + 1] = (float)(v / 16.0);
            o[3 * k + 2] = (float)(4.0 / r);
        }
        o[48] = (float)problem;
        o[49] = (float)(10.0 * area);
        for (int q = 0; q < 4; ++q) {
            const double R = std::min(radii[q], M_PI);
            int cnt = 0;
            for (const auto& pr : cand)
                if (pr.first <= R) cnt++;
            const double expect = std::max((N - 1) * 0.5 * (1.0 - std::cos(R)), 1e-12);
            o[50 + q] = (float)(cnt / expect);
        }
        o[54] = (float)(10.0 * (a[i] / amean - 1.0));
        o[55] = (float)amean;
    }
}

}  // namespace nce
