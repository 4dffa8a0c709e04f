// Host accuracy check of the FP64 logarithm (with its table) and Green's
// function used by the pair kernels (greens.hpp), against long-double
// references. Prints the largest errors in units of 2^-52 relative.
#include <cmath>
#include <cstdio>
#include <random>

#include "greens.hpp"

int main() {
    nce::LogEntry tab[nce::kLogTab];
    nce::build_log_table(tab);
    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    double worst_log = 0, worst_gi = 0, worst_ge = 0;
    for (int i = 0; i < 2000000; ++i) {
        double x = (i % 4 == 0) ? 1.0 + (U(g) - 0.5) * 1e-3 : std::exp(U(g) * std::log(1e7));
        long double ref = std::log((long double)x);
        double v = nce::log64t(x, tab);
        double err = std::fabs((long double)v - ref) / std::max(std::fabs((double)ref), 1e-300);
        if (std::fabs((double)ref) > 1e-3) worst_log = std::max(worst_log, err / 2.220446049250313e-16);
        double d = std::exp(std::log(1e-6) + U(g) * (std::log(2.0) - std::log(1e-6)));
        long double dl = d;
        long double gi = 2.0L / dl + std::log(2.0L / dl) - std::log1p(dl / 2.0L);
        long double ge = 2.0L / dl - std::log(2.0L / dl) - std::log1p(dl / 2.0L);
        worst_gi = std::max(worst_gi, (double)(std::fabs(nce::green64<0>(d * d, tab) - gi) / std::fabs(gi)) / 2.220446049250313e-16);
        worst_ge = std::max(worst_ge, (double)(std::fabs(nce::green64<1>(d * d, tab) - ge) / std::fabs(ge)) / 2.220446049250313e-16);
    }
    std::printf("log64 %.2f ulp, green interior %.2f ulp, green exterior %.2f ulp\n", worst_log, worst_gi, worst_ge);
    return (worst_log < 4 && worst_gi < 8 && worst_ge < 8) ? 0 : 1;
}
