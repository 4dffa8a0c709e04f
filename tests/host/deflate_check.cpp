// Host harness for the deflation basis (library host code, no GPU): reads N
// and N frames (9 numbers each); prints k, then the N x 16 basis row by row.
#include <cstdio>
#include <vector>

namespace nce {
// deflate_basis.cpp (declared in deflate.hpp, which also pulls in the HIP runtime)
int deflation_basis(const std::vector<double>& frames, int N, std::vector<double>& Z);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    int N;
    if (std::fscanf(f, "%d", &N) != 1) return 2;
    std::vector<double> fr((size_t)N * 9);
    for (auto& v : fr)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
    std::fclose(f);
    std::vector<double> Z;
    const int k = nce::deflation_basis(fr, N, Z);
    std::printf("%d\n", k);
    for (int i = 0; i < N; ++i) {
        for (int q = 0; q < 16; ++q) std::printf("%.17g ", Z[(size_t)i * 16 + q]);
        std::printf("\n");
    }
    return 0;
}
