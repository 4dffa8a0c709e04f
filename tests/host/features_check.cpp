// Host harness for the warm-start features (library host code, no GPU): reads
// N, eps, problem, then N frames (9 numbers) and N amplitudes; prints the
// N x 56 features, one patch per line.
#include <cstdint>
#include <cstdio>
#include <vector>

namespace nce {
// features.cpp (declared in mlp.hpp, which also pulls in the HIP runtime)
void patch_features(const std::vector<double>& frames, int64_t N, double eps, int problem,
                    const std::vector<double>& a, std::vector<float>& out);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    long N;
    double eps;
    int problem;
    if (std::fscanf(f, "%ld %lf %d", &N, &eps, &problem) != 3) return 2;
    std::vector<double> fr((size_t)N * 9), a((size_t)N);
    for (auto& v : fr)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
    for (auto& v : a)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
    std::fclose(f);
    std::vector<float> out;
    nce::patch_features(fr, N, eps, problem, a, out);
    for (long i = 0; i < N; ++i) {
        for (int k = 0; k < 56; ++k) std::printf("%.9g ", out[(size_t)i * 56 + k]);
        std::printf("\n");
    }
    return 0;
}
