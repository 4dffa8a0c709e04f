// Host check of the cube-sphere tree lists (library host code, no GPU):
// reads N centres (text), eps and the grid tolerance, builds the tree and
// verifies that every ordered pair of distinct patches is accounted for exactly
// once (direct list or one interpolated grid whose P2L sources contain it),
// that no patch sees itself, and that every grid lies in the far-field region
// of each of its sources, and that every P2L item's logarithm window holds the
// argument x of the item's pairs (x = u^2 + u interior, 1 + 1/u exterior, u
// half the chord) at the extreme configurations (grid point and skeleton point
// on the great circle through the two centres, nearest and farthest) and at
// random points of the cap and of the patch, for both problems, and that every
// P2L source uses the cheapest table of a synthetic recompression ladder that
// is valid over its grid's whole cap, a grid's sources sorted by table and at
// most kMaxTableRuns runs of one table per item. Prints "OK <stats>" or the
// first violation.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <cstdlib>
#include <random>
#include <vector>

#include "tree_build.hpp"

// the point at arclength r from unit vector c towards unit vector t (t not +-c)
static void toward(const double* c, const double* t, double r, double* out) {
    double d = c[0] * t[0] + c[1] * t[1] + c[2] * t[2];
    double e[3] = {t[0] - d * c[0], t[1] - d * c[1], t[2] - d * c[2]};
    const double n = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
    for (int k = 0; k < 3; ++k) out[k] = std::cos(r) * c[k] + std::sin(r) * e[k] / n;
}

// the point at arclength r from c in direction phi of the frame f (c, e1, e2)
static void around(const double* f, double r, double phi, double* out) {
    for (int k = 0; k < 3; ++k)
        out[k] = std::cos(r) * f[k] + std::sin(r) * (std::cos(phi) * f[3 + k] + std::sin(phi) * f[6 + k]);
}

static int octave_of(const double* p, const double* q, int problem) {
    const double dx = p[0] - q[0], dy = p[1] - q[1], dz = p[2] - q[2];
    const double u = 0.5 * std::sqrt(dx * dx + dy * dy + dz * dz);
    const double x = problem == 0 ? u * u + u : 1.0 + 1.0 / u;
    int e;
    std::frexp(x, &e);
    return e - 1;
}

// frame (c, e1, e2) of a unit vector
static void frame9(const double* c, double* f) {
    double a[3] = {0, 0, 1};
    if (std::fabs(c[2]) > 0.7) { a[0] = 1; a[2] = 0; }
    const double d = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    double e1[3] = {a[0] - d * c[0], a[1] - d * c[1], a[2] - d * c[2]};
    const double n = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double& v : e1) v /= n;
    const double e2[3] = {c[1] * e1[2] - c[2] * e1[1], c[2] * e1[0] - c[0] * e1[2], c[0] * e1[1] - c[1] * e1[0]};
    for (int k = 0; k < 3; ++k) { f[k] = c[k]; f[3 + k] = e1[k]; f[6 + k] = e2[k]; }
}

// every item's window against its pairs; returns false at the first miss
static bool check_windows(const nce::Tree& t, const std::vector<double>& fr, double eps, int problem) {
    if (t.it_win.size() != t.it_grid.size()) { std::printf("FAIL items without windows\n"); return false; }
    std::mt19937_64 g(11);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (size_t it = 0; it < t.it_grid.size(); ++it) {
        const int gi = t.it_grid[it], w0 = t.it_win[it];
        const double* gc = &t.g_frame[9 * gi];
        const double R = t.g_R[gi];
        for (int s = t.it_src0[it]; s < t.it_src1[it]; ++s) {
            const double* cj = &fr[9 * t.p2l_src[s]];
            double fj[9], p[3], q[3];
            frame9(cj, fj);
            int oct[6];
            toward(gc, cj, R, p);      // nearest pair
            toward(cj, gc, eps, q);
            oct[0] = octave_of(p, q, problem);
            toward(gc, cj, -R, p);     // farthest pair
            toward(cj, gc, -eps, q);
            oct[1] = octave_of(p, q, problem);
            for (int r = 2; r < 6; ++r) {
                around(&t.g_frame[9 * gi], R * std::sqrt(U(g)), 2 * M_PI * U(g), p);
                around(fj, eps * std::sqrt(U(g)), 2 * M_PI * U(g), q);
                oct[r] = octave_of(p, q, problem);
            }
            for (int o : oct)
                if (o < w0 || o >= w0 + nce::kLogWindowOctaves) {
                    std::printf("FAIL problem %d item %zu source %d: octave %d outside window %d..%d\n", problem, it,
                                t.p2l_src[s], o, w0, w0 + nce::kLogWindowOctaves - 1);
                    return false;
                }
        }
    }
    return true;
}

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
    // a ladder of recompressions valid beyond D_k = 2 eps 2^(k/2), smaller
    // with distance (two of equal size, as real ladders can have)
    for (int k = 1; k <= 12; ++k) {
        nce::FarTable ft;
        ft.D = 2.0 * eps * std::pow(2.0, 0.5 * k);
        ft.p = std::max(12, (int)(200 * std::pow(0.8, k)));
        tab.far.push_back(ft);
    }
    nce::Tree t;
    nce::build_tree(fr, N, eps, tab, tol, t);
    if (t.p2l_tab.size() != t.p2l_src.size()) { std::printf("FAIL sources without tables\n"); return 1; }
    for (size_t it = 0; it < t.it_grid.size(); ++it) {
        const int g = t.it_grid[it];
        int runs = 0;
        for (int s = t.it_src0[it]; s < t.it_src1[it]; ++s) {
            if (s == t.it_src0[it] || t.p2l_tab[s] != t.p2l_tab[s - 1]) ++runs;
            if (s > t.it_src0[it] && t.p2l_tab[s] < t.p2l_tab[s - 1]) { std::printf("FAIL item %zu not sorted by table\n", it); return 1; }
            const double* c = &fr[9 * t.p2l_src[s]];
            const double* gc = &t.g_frame[9 * g];
            double cr0 = c[1] * gc[2] - c[2] * gc[1], cr1 = c[2] * gc[0] - c[0] * gc[2], cr2 = c[0] * gc[1] - c[1] * gc[0];
            const double dm = std::atan2(std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2), c[0] * gc[0] + c[1] * gc[1] + c[2] * gc[2]) - t.g_R[g];
            const int k = t.p2l_tab[s];
            if (k > 0 && tab.far[k - 1].D > dm) { std::printf("FAIL source %d of grid %d: table %d not valid over the cap\n", t.p2l_src[s], g, k); return 1; }
            const int pk = k == 0 ? tab.p : tab.far[k - 1].p;
            for (size_t kk = 0; kk < tab.far.size(); ++kk)
                if (tab.far[kk].D <= dm && tab.far[kk].p < pk) { std::printf("FAIL source %d of grid %d: table %d not the cheapest\n", t.p2l_src[s], g, k); return 1; }
        }
        if (runs > nce::kMaxTableRuns) { std::printf("FAIL item %zu has %d table runs\n", it, runs); return 1; }
        if (it + 1 < t.it_grid.size() && t.it_grid[it + 1] == g && t.p2l_tab[t.it_src0[it + 1]] < t.p2l_tab[t.it_src1[it] - 1]) {
            std::printf("FAIL grid %d not sorted by table across items\n", g); return 1;
        }
    }
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
    for (int problem = 0; problem < 2; ++problem) {
        nce::PatchTables tp = tab;
        tp.problem = problem;
        nce::Tree tw;
        nce::build_tree(fr, N, eps, tp, tol, tw);
        if (!check_windows(tw, fr, eps, problem)) return 1;
    }
    // boxes with a second grid for their far sources: two consecutive grids
    // over the same cap, the second no larger than the first
    int split = 0;
    for (int g = 1; g < t.ngrid; ++g)
        if (t.g_R[g] == t.g_R[g - 1] && std::equal(&t.g_frame[9 * g], &t.g_frame[9 * g] + 9, &t.g_frame[9 * (g - 1)])) {
            ++split;
            if (t.g_nr[g] * t.g_nt[g] > t.g_nr[g - 1] * t.g_nt[g - 1]) { std::printf("FAIL far-source grid %d larger than its box's first\n", g); return 1; }
        }
    long maxdl = 0;
    for (long i = 0; i < N; ++i) maxdl = std::max(maxdl, (long)(t.dl_ptr[i + 1] - t.dl_ptr[i]));
    // FNV-1a over every array of the tree and its work counts: the build must
    // give the same bytes whatever the number of threads
    uint64_t h = 1469598103934665603ull;
    auto mix = [&h](const void* p, size_t n) {
        const unsigned char* b = static_cast<const unsigned char*>(p);
        for (size_t k = 0; k < n; ++k) h = (h ^ b[k]) * 1099511628211ull;
    };
    auto mixv = [&mix](const auto& v) { mix(v.data(), v.size() * sizeof(v[0])); };
    mixv(t.g_frame); mixv(t.g_R); mixv(t.g_nr); mixv(t.g_nt); mixv(t.g_level); mixv(t.g_table); mixv(t.g_off);
    mixv(t.g_item0); mixv(t.g_item1); mixv(t.it_grid); mixv(t.it_src0); mixv(t.it_src1); mixv(t.it_off);
    mixv(t.p2l_src); mixv(t.p2l_tab); mixv(t.it_win); mixv(t.dl_ptr); mixv(t.dl_src); mixv(t.l2t_ptr);
    mixv(t.l2t_grid);
    const double counts[3] = {t.pairs_far, t.pairs_near, t.interp_fma};
    mix(counts, sizeof(counts));
    std::printf("OK levels %d grids %d items %zu far %.4g near %.4g interp %.4g maxq %d maxdl %ld split %d hash %016llx\n",
                t.nlevels, t.ngrid, t.it_grid.size(), t.pairs_far, t.pairs_near, t.interp_fma, t.max_q, maxdl, split,
                (unsigned long long)h);
    return 0;
}
