// Green's function of the unit sphere restricted to the surface (Section 2.1,
// eqs. Gextonsurface and Gintonsurface) as used by every pair kernel. With the
// chord d and w = 2/d the two closed forms combine into one logarithm each:
//   exterior  2/d - log(2/d) - log(1 + d/2) = w - log(1 + w)
//   interior  2/d + log(2/d) - log(1 + d/2) = w + log(w^2 / (1 + w))
//
// FP64 logarithm (log64t): x = m 2^e with m in [1/2, 1); the top 10 bits of
// the mantissa pick a table entry (r_k, -log(2 r_k)) and v = m r_k - 1/2 =
// u / 2 with u = 2 m r_k - 1 (one fma, |u| < 2^-10.8), so log x = e ln 2 -
// log(2 r_k) + log(1 + u), the last by its degree-4 series (truncation below
// 2^-56 absolute), written in v as 2 (v - v^2 (1 - 4v/3 + 2v^2)) so that no
// fma needs two constants outside the inline set. r_k is an FP32 number
// within 2^-15 of the reciprocal of the bin centre of 2m, chosen (the
// accurate-tables idea of Gal's method) so that -log(2 r_k) lies within about
// 2^-62 of a double: one double then carries it, and an entry is 16 bytes
// read by one LDS instruction. The table is built on the host in extended
// precision; kernels stage it in LDS (16 KiB). Valid for positive normal
// arguments, which is all the kernels pass. Host builds of these functions
// serve the CPU accuracy test.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

namespace nce {

struct alignas(16) LogEntry {
    double t;  // -log(2 r_k), within about 2^-62 relative of the exact value
    double r;  // r_k
};
constexpr int kLogBits = 10;
constexpr int kLogTab = 1 << kLogBits;

// Host: fills the kLogTab entries. For each bin, among the FP32 numbers within
// 2^-15 of 1 / (bin centre), takes the one whose -log(2 r) is closest (in
// extended precision) to its own double rounding.
inline void build_log_table(LogEntry* tab) {
    for (int k = 0; k < kLogTab; ++k) {
        const long double c = 1.0L + (k + 0.5L) / kLogTab;
        const float r0 = (float)(1.0L / c);
        float best = r0;
        long double best_err = 1.0L;
        float r = r0;
        for (int j = 0; j < 512; ++j) r = std::nextafter(r, 0.0f);
        for (int j = -512; j <= 512; ++j, r = std::nextafter(r, 2.0f)) {
            const long double t = -std::log(2.0L * (long double)r);
            const long double err = std::fabs(t - (long double)(double)t) / std::fabs(t);
            if (err < best_err) {
                best_err = err;
                best = r;
            }
        }
        tab[k].t = (double)(-std::log(2.0L * (long double)best));
        tab[k].r = (double)best;
    }
}

// log x split as e ln 2 + t + 2 h: t = -log(2 r_k) from the table,
// 2 h = log(1 + u); de = e as a double.
struct LogParts {
    double t, h, de;
};
__host__ __device__ __forceinline__ LogParts log64t_parts(double x, const LogEntry* __restrict__ tab) {
    int e;
    double m;
#if defined(__HIP_DEVICE_COMPILE__)
    m = __builtin_amdgcn_frexp_mant(x);  // [1/2, 1)
    e = __builtin_amdgcn_frexp_exp(x);
    const unsigned hi = (unsigned)__double2hiint(m);
#else
    m = std::frexp(x, &e);
    unsigned long long bits;
    std::memcpy(&bits, &m, sizeof bits);
    const unsigned hi = (unsigned)(bits >> 32);
#endif
    // m and 2m share their mantissa bits: bin k of 2m in [1, 2)
    const LogEntry& L = tab[(hi >> (20 - kLogBits)) & (kLogTab - 1)];
    const double v = fma(m, L.r, -0.5);                         // u / 2, exact scaling
    const double q = fma(fma(v, 2.0, -4.0 / 3.0), v, 1.0);      // 1 - 4v/3 + 2v^2
    return {L.t, fma(-v * q, v, v), (double)e};
}

// log64t_parts with the series of log(1 + u) to degree 3: 2 (v - v^2 (1 - 4v/3)).
__host__ __device__ __forceinline__ LogParts log64t_parts3(double x, const LogEntry* __restrict__ tab) {
    int e;
    double m;
#if defined(__HIP_DEVICE_COMPILE__)
    m = __builtin_amdgcn_frexp_mant(x);
    e = __builtin_amdgcn_frexp_exp(x);
    const unsigned hi = (unsigned)__double2hiint(m);
#else
    m = std::frexp(x, &e);
    unsigned long long bits;
    std::memcpy(&bits, &m, sizeof bits);
    const unsigned hi = (unsigned)(bits >> 32);
#endif
    const LogEntry& L = tab[(hi >> (20 - kLogBits)) & (kLogTab - 1)];
    const double v = fma(m, L.r, -0.5);
    const double q = fma(v, -4.0 / 3.0, 1.0);
    return {L.t, fma(-v * q, v, v), (double)e};
}

// One first-order (Newton) correction of an estimate y of 1/sqrt(x):
// y (1 + e/2), e = 1 - x y^2; a relative error d of y becomes about -1.5 d^2.
__host__ __device__ __forceinline__ double rsqrt_first_order(double x, double y) {
    const double e = fma(-x * y, y, 1.0);
    return fma(y * 0.5, e, y);
}

// ln 2 = hi + lo with hi exact to 2^-32 so that e * hi is exact for |e| < 2^21
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;

__host__ __device__ __forceinline__ double log64t(double x, const LogEntry* __restrict__ tab) {
    const LogParts p = log64t_parts(x, tab);
    return fma(p.de, kLn2Hi, p.t) + fma(p.de, kLn2Lo, 2.0 * p.h);
}

// 1/sqrt(x) for positive normal x: the hardware estimate and one
// second-order correction y (1 + e/2 + 3e^2/8), e = 1 - x y^2 (no checks for
// zero, infinity or denormals, which no kernel passes).
__host__ __device__ __forceinline__ double rsqrt64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
#else
    return 1.0 / std::sqrt(x);
#endif
}

// G as a function of h2 = d^2 / 4, the squared half-distance (FP64). Then
// w = 2/d = 1/sqrt(h2) and u = 1/w = d/2 = h2 w, and the interior logarithm
// log(w^2 / (1 + w)) = -log(u^2 + u) needs no division. The pair kernels keep
// coordinates pre-scaled by 1/2 (exact), so h2 comes straight from them.
template <int PROB>
__host__ __device__ __forceinline__ double green64_half(double h2, const LogEntry* __restrict__ tab) {
    const double w = rsqrt64(h2);
    if (PROB == 1) return w - log64t(1.0 + w, tab);
    const double u = h2 * w;
    return w - log64t(fma(u, u, u), tab);
}

// G = g - e ln 2 (FP64) with e the binary exponent of the logarithm's
// argument, returned separately (de) so that a sum over many pairs can carry
// sum rho e apart from sum rho g and apply ln 2 once at the end: per pair this
// saves the conversion of e ln 2 into the logarithm.
template <int PROB>
__host__ __device__ __forceinline__ double green64_half_split(double h2, const LogEntry* __restrict__ tab,
                                                              double& de) {
    const double w = rsqrt64(h2);
    double x;
    if (PROB == 1) {
        x = 1.0 + w;
    } else {
        const double u = h2 * w;
        x = fma(u, u, u);
    }
    const LogParts p = log64t_parts(x, tab);
    de = p.de;
    return fma(-2.0, p.h, w - p.t);
}

// The same split form at the precision of the incoming grids, which
// interpolate the far field to tol_grid (1e-8 by default) and so gain nothing
// from full double precision per pair: a first-order correction of the
// hardware reciprocal square root (its estimate is within 2^-24.2 relative
// over [1e-9, 3] on gfx950, the corrected value within 2^-47.8, measured) and
// the logarithm's series to degree 3 (truncation 2 v^4 below 2^-46.2
// absolute). Two FP64 operations fewer per pair than green64_half_split.
__host__ __device__ __forceinline__ double rsqrt64_grid(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y = __builtin_amdgcn_rsq(x);
    return rsqrt_first_order(x, y);
#else
    return 1.0 / std::sqrt(x);
#endif
}

template <int PROB>
__host__ __device__ __forceinline__ double green64_grid_split(double h2, const LogEntry* __restrict__ tab,
                                                              double& de) {
    const double w = rsqrt64_grid(h2);
    double x;
    if (PROB == 1) {
        x = 1.0 + w;
    } else {
        const double u = h2 * w;
        x = fma(u, u, u);
    }
    const LogParts p = log64t_parts3(x, tab);
    de = p.de;
    return fma(-2.0, p.h, w - p.t);
}

// The grid form with the logarithm's binary exponent folded into its table.
// A window of kWinOct consecutive octaves of the argument x, x in [2^E0,
// 2^(E0 + kWinOct)), kWinBins bins per octave, is indexed straight by the high
// word of x: the low kWinOctBits bits of the biased exponent and the top
// kWinBinBits bits of the mantissa (octave E sits in slot (E + 1023) mod
// kWinOct). The entry of bin k of octave E is r = r_k 2^-(E+1), with r_k the
// double nearest 1 / c_k, c_k = 1 + (k + 1/2) / kWinBins the bin centre, and
// t = E ln 2 - log(r_k) rounded once: then v = x r - 1/2 lies within
// 2^-(kWinBinBits + 2) of zero, log x = t + log(1 + 2 v), and the
// series of log(1 + 2 v) / 2 to degree 4 leaves under 2^-48 absolute. Against
// the split form this drops the exponent's extraction and conversion and its
// second accumulator, for one more series term. The caller guarantees x in
// the window for every pair of nonzero strength (an index outside it reads
// another octave's entry: a finite wrong value).
constexpr int kWinOctBits = 3;
constexpr int kWinBinBits = 8;
constexpr int kWinOct = 1 << kWinOctBits;
constexpr int kWinBins = 1 << kWinBinBits;
constexpr int kWinTab = kWinOct * kWinBins;

// Host: entries of octaves e_first .. e_first + noct - 1, noct x kWinBins.
inline void build_log_window_table(int e_first, int noct, LogEntry* tab) {
    const long double ln2 = 0.693147180559945309417232121458176568L;
    for (int k = 0; k < kWinBins; ++k) {
        const long double c = 1.0L + (k + 0.5L) / kWinBins;
        const double rk = (double)(1.0L / c);
        const long double base = -std::log((long double)rk);
        for (int o = 0; o < noct; ++o) {
            const int e = e_first + o;
            tab[(size_t)o * kWinBins + k].r = std::ldexp(rk, -(e + 1));
            tab[(size_t)o * kWinBins + k].t = (double)(base + (long double)e * ln2);
        }
    }
}

// The octave held by slot `slot` of the window that starts at octave e0.
__host__ __device__ __forceinline__ int window_octave(int e0, int slot) {
    return e0 + ((slot - e0 - 1023) & (kWinOct - 1));
}

// The windowed grid form in the argument s = d^2 / 16 (the pair kernel keeps
// its coordinates quarter-scaled, exact), given an estimate y0 of 1 / sqrt(s)
// within about 2^-24 relative. One Newton step for 1 / sqrt(s) is
// y0 (3 - s y0^2) / 2, and 1 / sqrt(s) = 4 / d = 2 w, so W = y0 (3 - p y0)
// with p = s y0 is 4 w, the first-order corrected w = 2 / d scaled by four,
// and u = d / 2 = s W = p (3 - p y0): three operations where the
// correction of an estimate of w takes four before u. The 1/4 rides on the
// fma that subtracts the table's t. The logarithm's series is taken in
// Horner form: log(1 + 2v) = 2v - 2v^2 + (8/3) v^3 - 4 v^4 is
// -v (v (2 - (8/3) v + 4 v^2) - 2), two fmas and no separate multiply after
// its quadratic factor. x (u^2 + u, or 1 + w) and so the window are those of
// the half-distance form.
template <int PROB>
__host__ __device__ __forceinline__ double green64_quarter_win(double s, double y0, const LogEntry* __restrict__ win) {
    const double p = s * y0;
    const double t = fma(-p, y0, 3.0);
    const double W = y0 * t;  // 4 w
    double x;
    if (PROB == 1) {
        x = fma(W, 0.25, 1.0);
    } else {
        const double u = p * t;
        x = fma(u, u, u);
    }
#if defined(__HIP_DEVICE_COMPILE__)
    const unsigned hi = (unsigned)__double2hiint(x);
#else
    unsigned long long bits;
    std::memcpy(&bits, &x, sizeof bits);
    const unsigned hi = (unsigned)(bits >> 32);
#endif
    const LogEntry& L = win[(hi >> (20 - kWinBinBits)) & (kWinTab - 1)];
    const double v = fma(x, L.r, -0.5);
    const double q2 = fma(fma(v, 4.0, -8.0 / 3.0), v, 2.0);
    return fma(v, fma(v, q2, -2.0), fma(W, 0.25, -L.t));
}

// The same with the estimate of 1 / sqrt(s) taken here: the hardware's on the
// device, the exact value on the host.
template <int PROB>
__host__ __device__ __forceinline__ double green64_grid_win(double s, const LogEntry* __restrict__ win) {
#if defined(__HIP_DEVICE_COMPILE__)
    const double y0 = __builtin_amdgcn_rsq(s);
#else
    const double y0 = 1.0 / std::sqrt(s);
#endif
    return green64_quarter_win<PROB>(s, y0, win);
}

// G as a function of d^2 (FP64).
template <int PROB>
__host__ __device__ __forceinline__ double green64(double d2, const LogEntry* __restrict__ tab) {
    return green64_half<PROB>(0.25 * d2, tab);
}

#if defined(__HIPCC__)
// FP32: hardware reciprocal square root and base-2 logarithm (two
// transcendentals per pair). The two parts are returned separately,
// G = w - ln2 l2, so the caller folds the ln 2 scale into its accumulator:
// exterior l2 = log2(1 + w); interior l2 = log2(u^2 + u), u = d/2 (as green64).
// Argument h2 = d^2 / 4 as for green64_half.
template <int PROB>
__device__ __forceinline__ void green32_parts_half(float h2, float& w, float& l2) {
    w = __builtin_amdgcn_rsqf(h2);
    if (PROB == 1) {
        l2 = __builtin_amdgcn_logf(1.0f + w);
    } else {
        const float u = h2 * w;
        l2 = __builtin_amdgcn_logf(fmaf(u, u, u));
    }
}
#endif

}  // namespace nce
