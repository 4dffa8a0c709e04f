// Host check of the cube-sphere tree lists (library host code, no GPU):
// reads N centres (text), eps and the grid tolerance, builds the tree and
// verifies that every ordered pair of distinct patches is accounted for exactly
// once (direct list or one interpolated grid whose P2L sources contain it),
// that no patch sees itself, and that every grid lies in the far-field region
// of each of its sources. Prints "OK <stats>" or the first violation.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tree_build.hpp"

int main(int argc, char** argv) {
    if (argc < 4) return 2;
    FILE* f = std::fopen(argv[1], "r");
    double eps = std::atof(argv[2]), tol = std::atof(argv[3]);
    long N;
    if (std::fscanf(f, "%ld", &N) != 1) return 2;
    std::vector<double> fr(N * 9, 0.0);
    for (long i = 0; i < N; ++i)
        if (std::fscanf(f, "%lf %lf %lf", &fr[9 * i], &fr[9 * i + 1], &fr[9 * i + 2]) != 3) return 2;
    std::fclose(f);
    nce::PatchTables tab;
    tab.Kstar = 512;
    tab.p = 200;
    nce::Tree t;
    nce::build_tree(fr, N, eps, tab, tol, t);
    // grid -> set of sources
    std::vector<std::vector<int>> gsrc(t.ngrid);
    for (size_t it = 0; it < t.it_grid.size(); ++it)
        for (int s = t.it_src0[it]; s < t.it_src1[it]; ++s) gsrc[t.it_grid[it]].push_back(t.p2l_src[s]);
    std::vector<int> cnt(N);
    for (long i = 0; i < N; ++i) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (long q = t.dl_ptr[i]; q < t.dl_ptr[i + 1]; ++q) cnt[t.dl_src[q]]++;
        for (long q = t.l2t_ptr[i]; q < t.l2t_ptr[i + 1]; ++q) {
            int g = t.l2t_grid[q];
            for (int j : gsrc[g]) cnt[j]++;
            // member inside the cap
            const double* c = &fr[9 * i];
            const double* gc = &t.g_frame[9 * g];
            double cr0 = c[1] * gc[2] - c[2] * gc[1], cr1 = c[2] * gc[0] - c[0] * gc[2], cr2 = c[0] * gc[1] - c[1] * gc[0];
            double d = std::atan2(std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2), c[0] * gc[0] + c[1] * gc[1] + c[2] * gc[2]);
            if (d + eps > t.g_R[g] * (1 + 1e-12)) { std::printf("FAIL member %ld outside cap %d\n", i, g); return 1; }
        }
        for (long j = 0; j < N; ++j) {
            int want = (j == i) ? 0 : 1;
            if (cnt[j] != want) { std::printf("FAIL pair (%ld,%ld) counted %d times\n", i, j, cnt[j]); return 1; }
        }
    }
    for (int g = 0; g < t.ngrid; ++g)
        for (int j : gsrc[g]) {
            const double* c = &fr[9 * j];
            const double* gc = &t.g_frame[9 * g];
            double cr0 = c[1] * gc[2] - c[2] * gc[1], cr1 = c[2] * gc[0] - c[0] * gc[2], cr2 = c[0] * gc[1] - c[1] * gc[0];
            double d = std::atan2(std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2), c[0] * gc[0] + c[1] * gc[1] + c[2] * gc[2]);
            if (d - t.g_R[g] <= 2 * eps) { std::printf("FAIL grid %d not in far field of %d\n", g, j); return 1; }
        }
    long maxdl = 0;
    for (long i = 0; i < N; ++i) maxdl = std::max(maxdl, (long)(t.dl_ptr[i + 1] - t.dl_ptr[i]));
    std::printf("OK levels %d grids %d items %zu far %.4g near %.4g interp %.4g maxq %d maxdl %ld\n", t.nlevels,
                t.ngrid, t.it_grid.size(), t.pairs_far, t.pairs_near, t.interp_fma, t.max_q, maxdl);
    return 0;
}
