// Green's function of the unit sphere restricted to the surface (Section 2.1,
// eqs. Gextonsurface and Gintonsurface) as used by every pair kernel. With the
// chord d and w = 2/d the two closed forms combine into one logarithm each:
//   exterior  2/d - log(2/d) - log(1 + d/2) = w - log(1 + w)
//   interior  2/d + log(2/d) - log(1 + d/2) = w + log(w^2 / (1 + w))
//
// The FP64 logarithm is a short table-free routine: x = m 2^e with m in
// [sqrt(1/2), sqrt(2)), log m = 2 atanh(u), u = (m - 1)/(m + 1), |u| <= 0.1716,
// summed as the odd series 2u (1 + u^2/3 + ... + u^20/21) (truncation below
// 2^-53 relative), and e ln 2 added with a two-part ln 2. It is valid for
// positive normal arguments, which is all the kernels pass (w >= 1). The
// quotient and the reciprocal use the hardware reciprocal with Newton steps.
// Host builds of these functions exist only for the CPU accuracy test.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace nce {

__host__ __device__ __forceinline__ double rcp64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r = __builtin_amdgcn_rcp(x);
#else
    double r = (double)(1.0f / (float)x);  // same starting accuracy class as the hardware estimate
#endif
    // two Newton steps: r (2 - x r)
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    return r;
}

// a / b to about one ulp (reciprocal, then one residual correction)
__host__ __device__ __forceinline__ double div64(double a, double b) {
    const double r = rcp64(b);
    const double q = a * r;
    return fma(fma(-b, q, a), r, q);
}

__host__ __device__ __forceinline__ double log64(double x) {
    int e;
#if defined(__HIP_DEVICE_COMPILE__)
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    e = __builtin_amdgcn_frexp_exp(x);
#else
    double m = std::frexp(x, &e);
#endif
    if (m < 0.70710678118654752440) {
        m *= 2.0;
        e -= 1;
    }
    const double u = div64(m - 1.0, m + 1.0);
    const double s = u * u;
    double p = 1.0 / 21.0;
    p = fma(p, s, 1.0 / 19.0);
    p = fma(p, s, 1.0 / 17.0);
    p = fma(p, s, 1.0 / 15.0);
    p = fma(p, s, 1.0 / 13.0);
    p = fma(p, s, 1.0 / 11.0);
    p = fma(p, s, 1.0 / 9.0);
    p = fma(p, s, 1.0 / 7.0);
    p = fma(p, s, 1.0 / 5.0);
    p = fma(p, s, 1.0 / 3.0);
    const double lm = fma(2.0 * u * s, p, 2.0 * u);  // 2u + 2u s P(s)
    const double de = (double)e;
    // ln 2 = hi + lo with hi exact to 2^-32 so that e * hi is exact for |e| < 2^21
    const double ln2_hi = 6.93147180369123816490e-01;
    const double ln2_lo = 1.90821492927058770002e-10;
    return fma(de, ln2_hi, fma(de, ln2_lo, lm));
}

__host__ __device__ __forceinline__ double rsqrt64(double x) {
#if defined(__HIP_DEVICE_COMPILE__)
    return rsqrt(x);
#else
    return 1.0 / std::sqrt(x);
#endif
}

// G as a function of h2 = d^2 / 4, the squared half-distance (FP64). Then
// w = 2/d = 1/sqrt(h2) and u = 1/w = d/2 = h2 w, and the interior logarithm
// log(w^2 / (1 + w)) = -log(u^2 + u) needs no division. The pair kernels keep
// coordinates pre-scaled by 1/2 (exact), so h2 comes straight from them.
template <int PROB>
__host__ __device__ __forceinline__ double green64_half(double h2) {
    const double w = rsqrt64(h2);
    if (PROB == 1) return w - log64(1.0 + w);
    const double u = h2 * w;
    return w - log64(fma(u, u, u));
}

// G as a function of d^2 (FP64).
template <int PROB>
__host__ __device__ __forceinline__ double green64(double d2) {
    return green64_half<PROB>(0.25 * d2);
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
