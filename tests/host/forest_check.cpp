// Host check of a forest (several independent configurations in one patch
// numbering, library host code, no GPU): reads B configurations (text: B, then
// per configuration N and N centres), eps and the grid tolerance; builds every
// configuration's tree (every third configuration summed directly instead),
// appends them, and verifies for every target patch that each other patch of
// its own configuration is accounted for exactly once (direct list or one
// grid whose P2L sources contain it), that no patch of another configuration
// and not the patch itself appears, and that the configuration index of every
// item, grid and patch is the one it came from. Prints "OK <stats>" or the
// first violation.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tree_build.hpp"

int main(int argc, char** argv) {
    if (argc < 4) return 2;
    FILE* f = std::fopen(argv[1], "r");
    const double eps = std::atof(argv[2]), tol = std::atof(argv[3]);
    int B;
    if (std::fscanf(f, "%d", &B) != 1) return 2;
    std::vector<std::vector<double>> fr(B);
    std::vector<long> first{0};
    for (int b = 0; b < B; ++b) {
        long N;
        if (std::fscanf(f, "%ld", &N) != 1) return 2;
        fr[b].assign(N * 9, 0.0);
        for (long i = 0; i < N; ++i)
            if (std::fscanf(f, "%lf %lf %lf", &fr[b][9 * i], &fr[b][9 * i + 1], &fr[b][9 * i + 2]) != 3) return 2;
        first.push_back(first.back() + N);
    }
    std::fclose(f);
    nce::PatchTables tab;
    tab.Kstar = 512;
    tab.p = 200;
    nce::Tree forest;
    nce::start_forest(forest);
    for (int b = 0; b < B; ++b) {
        const long N = first[b + 1] - first[b];
        if (b % 3 == 2 || N < 2) {
            nce::append_direct(forest, first[b], N, tab.Kstar, tab.p);
        } else {
            nce::Tree t;
            nce::build_tree(fr[b], N, eps, tab, tol, t);
            nce::append_tree(forest, t, first[b]);
        }
    }
    const long NT = first.back();
    if (forest.N != NT || (long)forest.dl_ptr.size() != NT + 1 || (long)forest.l2t_ptr.size() != NT + 1 ||
        (long)forest.pt_cfg.size() != NT || forest.ncfg != B) {
        std::printf("FAIL sizes\n");
        return 1;
    }
    std::vector<int> cfg_of(NT);
    for (int b = 0; b < B; ++b)
        for (long i = first[b]; i < first[b + 1]; ++i) cfg_of[i] = b;
    for (long i = 0; i < NT; ++i)
        if (forest.pt_cfg[i] != cfg_of[i]) { std::printf("FAIL pt_cfg %ld\n", i); return 1; }
    std::vector<std::vector<int>> gsrc(forest.ngrid);
    for (size_t it = 0; it < forest.it_grid.size(); ++it) {
        const int g = forest.it_grid[it];
        if (forest.it_cfg[it] != forest.g_cfg[g]) { std::printf("FAIL it_cfg %zu\n", it); return 1; }
        for (int s = forest.it_src0[it]; s < forest.it_src1[it]; ++s) {
            const int j = forest.p2l_src[s];
            if (cfg_of[j] != forest.g_cfg[g]) { std::printf("FAIL grid %d source %d from another configuration\n", g, j); return 1; }
            gsrc[g].push_back(j);
        }
    }
    std::vector<int> cnt(NT);
    for (long i = 0; i < NT; ++i) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (long q = forest.dl_ptr[i]; q < forest.dl_ptr[i + 1]; ++q) cnt[forest.dl_src[q]]++;
        for (long q = forest.l2t_ptr[i]; q < forest.l2t_ptr[i + 1]; ++q) {
            const int g = forest.l2t_grid[q];
            if (forest.g_cfg[g] != cfg_of[i]) { std::printf("FAIL patch %ld reads a grid of another configuration\n", i); return 1; }
            for (int j : gsrc[g]) cnt[j]++;
        }
        for (long j = 0; j < NT; ++j) {
            const int want = (j != i && cfg_of[j] == cfg_of[i]) ? 1 : 0;
            if (cnt[j] != want) { std::printf("FAIL pair (%ld,%ld) counted %d times\n", i, j, cnt[j]); return 1; }
        }
    }
    if (forest.it_win.size() != forest.it_grid.size() || forest.p2l_tab.size() != forest.p2l_src.size()) {
        std::printf("FAIL the forest lost its items' logarithm windows or sources' tables\n");
        return 1;
    }
    std::printf("OK configurations %d patches %ld grids %d items %zu far %.4g near %.4g\n", B, NT, forest.ngrid,
                forest.it_grid.size(), forest.pairs_far, forest.pairs_near);
    return 0;
}
