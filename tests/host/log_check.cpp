// Host accuracy check of the FP64 logarithm (with its table) and Green's
// function used by the pair kernels (greens.hpp), against long-double
// references. Prints the largest errors in units of 2^-52: relative for the
// Green's functions; for the logarithm relative to max(|log x|, 1/2), since
// it only enters G = w -+ log(..), whose terms are at least 1/2 in size (its
// series leaves up to 2^-56 absolute near x = 1).
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "greens.hpp"

// The window of octaves e0 .. e0 + kWinOct - 1 as the far-field kernel loads it
// from the table of octaves e_first .. (slot s of the window: octave
// window_octave(e0, s)).
static void load_window(const std::vector<nce::LogEntry>& all, int e_first, int e0, nce::LogEntry* win) {
    for (int k = 0; k < nce::kWinTab; ++k) {
        const int e = nce::window_octave(e0, k >> nce::kWinBinBits);
        win[k] = all[(size_t)(e - e_first) * nce::kWinBins + (k & (nce::kWinBins - 1))];
    }
}

int main() {
    static nce::LogEntry tab[nce::kLogTab];
    nce::build_log_table(tab);
    // octaves -60 .. 60 of the windowed table
    const int e_first = -60, noct = 121;
    std::vector<nce::LogEntry> wall((size_t)noct * nce::kWinBins);
    nce::build_log_window_table(e_first, noct, wall.data());
    static nce::LogEntry win[nce::kWinTab];
    double worst_win = 0;
    int bad_slot = 0;
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double worst_log = 0, worst_gi = 0, worst_ge = 0, worst_si = 0, worst_se = 0, worst_grid = 0, worst_rsq = 0;
    for (int i = 0; i < 2000000; ++i) {
        double x = (i % 4 == 0) ? 1.0 + (U(g) - 0.5) * 1e-3 : std::exp(U(g) * std::log(1e7));
        long double ref = std::log((long double)x);
        double v = nce::log64t(x, tab);
        double err = std::fabs((long double)v - ref) / std::max(std::fabs((double)ref), 0.5);
        worst_log = std::max(worst_log, err / 2.220446049250313e-16);
        double d = std::exp(std::log(1e-6) + U(g) * (std::log(2.0) - std::log(1e-6)));
        long double dl = d;
        long double gi = 2.0L / dl + std::log(2.0L / dl) - std::log1p(dl / 2.0L);
        long double ge = 2.0L / dl - std::log(2.0L / dl) - std::log1p(dl / 2.0L);
        worst_gi = std::max(worst_gi, (double)(std::fabs(nce::green64<0>(d * d, tab) - gi) / std::fabs(gi)) / 2.220446049250313e-16);
        worst_ge = std::max(worst_ge, (double)(std::fabs(nce::green64<1>(d * d, tab) - ge) / std::fabs(ge)) / 2.220446049250313e-16);
        // the split form the far-field sums carry: G = g - e ln 2
        double de;
        const double si = nce::green64_half_split<0>(0.25 * d * d, tab, de);
        const double vi = std::fma(-nce::kLn2Hi, de, std::fma(-nce::kLn2Lo, de, si));
        const double se = nce::green64_half_split<1>(0.25 * d * d, tab, de);
        const double ve = std::fma(-nce::kLn2Hi, de, std::fma(-nce::kLn2Lo, de, se));
        worst_si = std::max(worst_si, (double)(std::fabs(vi - gi) / std::fabs(gi)) / 2.220446049250313e-16);
        worst_se = std::max(worst_se, (double)(std::fabs(ve - ge) / std::fabs(ge)) / 2.220446049250313e-16);
        // the far-field grid form (degree-3 series): absolute error of G
        // against 2^-44 (the host build takes an exact rsqrt)
        for (int prob = 0; prob < 2; ++prob) {
            const double sg = prob ? nce::green64_grid_split<1>(0.25 * d * d, tab, de)
                                   : nce::green64_grid_split<0>(0.25 * d * d, tab, de);
            const double vg = std::fma(-nce::kLn2Hi, de, std::fma(-nce::kLn2Lo, de, sg));
            const long double ref = prob ? ge : gi;
            worst_grid = std::max(worst_grid, (double)(std::fabs(vg - ref) / std::max(std::fabs(ref), 1.0L)));
        }
        // the windowed grid form: a window holding x's octave at a random slot
        // (every slot is hit), absolute error of G against 2^-44
        for (int prob = 0; prob < 2; ++prob) {
            const double hh = 0.25 * d * d, w = 1.0 / std::sqrt(hh);
            const double x = prob ? 1.0 + w : std::fma(hh * w, hh * w, hh * w);
            int ex;
            std::frexp(x, &ex);   // x in [2^(ex-1), 2^ex)
            const int e0 = (ex - 1) - (int)(U(g) * nce::kWinOct);
            load_window(wall, e_first, e0, win);
            // the slot the index picks holds x's own octave
            unsigned long long bits;
            std::memcpy(&bits, &x, sizeof bits);
            const int slot = (int)((bits >> 52) & (nce::kWinOct - 1));
            if (nce::window_octave(e0, slot) != ex - 1) ++bad_slot;
            // the kernel's argument is s = d^2 / 16; its estimate of 1 / sqrt(s)
            // exact (the host build) and off by the largest error measured
            // for the gfx950 FP64 rsq (2^-24.2), either sign
            const double sq = 0.0625 * d * d;
            const double vg = prob ? nce::green64_grid_win<1>(sq, win) : nce::green64_grid_win<0>(sq, win);
            const long double ref = prob ? ge : gi;
            worst_win = std::max(worst_win, (double)(std::fabs(vg - ref) / std::max(std::fabs(ref), 1.0L)));
            const long double rs = 1.0L / std::sqrt((long double)sq);
            for (int sgn = -1; sgn <= 1; sgn += 2) {
                const double y0 = (double)(rs * (1.0L + sgn * 5.2e-8L));
                const double vq = prob ? nce::green64_quarter_win<1>(sq, y0, win) : nce::green64_quarter_win<0>(sq, y0, win);
                worst_win = std::max(worst_win, (double)(std::fabs(vq - ref) / std::max(std::fabs(ref), 1.0L)));
            }
        }
        // first-order correction of an estimate at the largest error measured
        // for the gfx950 FP64 rsq (2^-24.2), either sign: about 1.5 d^2
        const double h2 = 0.25 * d * d;
        const long double r = 1.0L / std::sqrt((long double)h2);
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            const double y0 = (double)(r * (1.0L + sgn * 5.2e-8L));
            const double y1 = nce::rsqrt_first_order(h2, y0);
            worst_rsq = std::max(worst_rsq, (double)std::fabs(y1 / r - 1.0L));
        }
    }
    std::printf("log64 %.2f ulp, green interior %.2f ulp, green exterior %.2f ulp, split %.2f / %.2f ulp\n", worst_log,
                worst_gi, worst_ge, worst_si, worst_se);
    std::printf("grid form: G within %.3e (abs, or rel above 1); first-order rsq correction within %.3e\n", worst_grid,
                worst_rsq);
    std::printf("windowed grid form: G within %.3e; windows whose indexed slot missed x's octave: %d\n", worst_win,
                bad_slot);
    return (worst_log < 4 && worst_gi < 6 && worst_ge < 6 && worst_si < 8 && worst_se < 8 &&
            worst_grid < std::ldexp(1.0, -44) && worst_rsq < 5e-15 && worst_win < std::ldexp(1.0, -44) &&
            bad_slot == 0)
               ? 0
               : 1;
}
