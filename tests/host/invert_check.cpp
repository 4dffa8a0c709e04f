// Host harness for the deflation's coarse-matrix inversion (library host code,
// no GPU): reads k and a k x k matrix T (row-major); prints "ok" and
// M = T^{-1} - I as 16 x 16 (zero beyond k), or "singular".
#include <cstdio>
#include <vector>

namespace nce {
// deflate_basis.cpp (declared in deflate.hpp, which also pulls in the HIP runtime)
bool deflation_invert(std::vector<double> T, int k, std::vector<double>& M);
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    FILE* f = std::fopen(argv[1], "r");
    int k;
    if (std::fscanf(f, "%d", &k) != 1) return 2;
    std::vector<double> T((size_t)k * k);
    for (auto& v : T)
        if (std::fscanf(f, "%lf", &v) != 1) return 2;
    std::fclose(f);
    std::vector<double> M;
    if (!nce::deflation_invert(T, k, M)) {
        std::printf("singular\n");
        return 0;
    }
    std::printf("ok\n");
    for (int a = 0; a < 16; ++a) {
        for (int b = 0; b < 16; ++b) std::printf("%.17g ", M[(size_t)a * 16 + b]);
        std::printf("\n");
    }
    return 0;
}
