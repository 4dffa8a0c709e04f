// Field of the patch densities at points of the domain (Sections 2.2 and 2.3)
// and the L2 residual of the absorbing condition on a patch (eq. l2res).
//
// The potential at a target x is the sum over patches j of the integral of
// G(x, x') sigma_j(x') over patch j, G the off-surface Neumann Green's
// function (eqs. Gextoffsurface, Gintoffsurface), sigma_j = B f_j:
//   * patches whose centre lies at arclength >= 3 eps from x/|x|: the
//     compressed outgoing representation, sum_m G(x, s_jm) rho_jm with
//     rho_j = T f_j (Section 7.1; the same skeleton as the system apply);
//   * nearer patches: quadrature of sigma_j itself, the one-patch solve's
//     radial rule (13 panels x 20 nodes, the Jacobi factor on the last) times
//     kNearTheta equispaced angles; sigma_j's angular dependence is a
//     trigonometric polynomial of degree M, evaluated from its Fourier
//     coefficients per radial node;
//   * a target on the sphere inside patch i: patch i's term is the patch data
//     sum_k f_ik Z_k(t/eps, theta), which the one-patch solution reproduces on
//     its own patch (Section 9).
// The physical fields are ubar = 1 - u (exterior) and vbar = (v - 1)/(3 D) +
// (1 - |x|^2)/6 with D = -I_sigma (interior, eq. vtilde).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"

using namespace nce_detail;

namespace nce {
namespace {

constexpr int kNearTheta = 256;   // angles of the near-patch quadrature (one per thread)
constexpr int kNearChunk = 64;    // radial nodes per LDS pass of the near kernel
constexpr int kFarStage = 512;    // skeleton points staged per LDS pass
constexpr int kMaxModes = 16;     // M <= 15

// G(x, y) for y on the unit sphere and x in the domain (|x| = r; h = x / r,
// or 0 at the origin), from coordinate differences: d = |x - y|,
// s2 = |h - y|^2, a = 1 - x.y = (1 - r) + r s2 / 2.
//   interior (r <= 1): 2/d + log(2 / (a + d))
//   exterior (r >= 1): 2/d + log((r - x.y) / (a + d)), r - x.y = r s2 / 2;
//     when a <= 0 the same ratio as (d - a) / (r (1 + cos)), since
//     (a + d)(d - a) = r^2 sin^2, and 1 + cos = 2 - s2 / 2.
template <int PROB>
__device__ __forceinline__ double green_off(double dx, double dy, double dz, double ex, double ey, double ez,
                                            double r) {
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double s2 = ex * ex + ey * ey + ez * ez;
    const double a = (1.0 - r) + 0.5 * r * s2;
    double lg;
    if (PROB == 0)
        lg = log(2.0 / (a + d));
    else if (a > 0.0)
        lg = log(0.5 * r * s2 / (a + d));
    else
        lg = log((d - a) / (r * (2.0 - 0.5 * s2)));
    return 2.0 / d + lg;
}

// Far part: one thread per target, blocks over (targets, patch chunks); the
// skeleton points of each source patch are staged in LDS. Targets skip the
// patches of their own skip list (near patches and the patch they lie on),
// sorted by patch index: skip[sptr[t] .. sptr[t+1]).
// Several radii (ptype non-null): source j uses its radius's base skeleton
// (t_p[ptype[j] ntab] points from skeleton index t_soff[ptype[j] ntab]);
// strengths rho have rows of ldr.
template <int PROB>
__global__ __launch_bounds__(256) void k_field_far(int64_t n, const double4* __restrict__ pts, int N, int p,
                                                   const double* __restrict__ frames,
                                                   const double* __restrict__ skel_off,
                                                   const double* __restrict__ rho, int ldr,
                                                   const int64_t* __restrict__ sptr, const int* __restrict__ skip,
                                                   int chunk, double* __restrict__ partial,
                                                   const int* __restrict__ ptype, const int* __restrict__ t_soff,
                                                   const int* __restrict__ t_p, int ntab) {
    __shared__ double4 sm[kFarStage];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool act = t < n;
    const double4 P = act ? pts[t] : make_double4(0.0, 0.0, 0.0, 0.0);
    const double r = P.w;
    const double hs = r > 0.0 ? 1.0 / r : 0.0;
    const double hx = P.x * hs, hy = P.y * hs, hz = P.z * hs;
    int64_t q = act ? sptr[t] : 0;
    const int64_t qe = act ? sptr[t + 1] : 0;
    const int j0 = blockIdx.y * chunk, j1 = min(N, j0 + chunk);
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
        while (q < qe && skip[q] < j) ++q;
        const bool use = act && !(q < qe && skip[q] == j);
        const double* f = frames + 9 * (int64_t)j;
        const int pj = ptype ? t_p[ptype[j] * ntab] : p;
        const double* so = ptype ? skel_off + 3 * (int64_t)t_soff[ptype[j] * ntab] : skel_off;
        for (int m0 = 0; m0 < pj; m0 += kFarStage) {
            const int cnt = min(kFarStage, pj - m0);
            __syncthreads();
            for (int m = threadIdx.x; m < cnt; m += 256) {
                const double* o = so + 3 * (m0 + m);
                double4 v;
                v.x = f[0] + (o[0] * f[0] + o[1] * f[3] + o[2] * f[6]);
                v.y = f[1] + (o[0] * f[1] + o[1] * f[4] + o[2] * f[7]);
                v.z = f[2] + (o[0] * f[2] + o[1] * f[5] + o[2] * f[8]);
                v.w = rho[(int64_t)j * ldr + m0 + m];
                sm[m] = v;
            }
            __syncthreads();
            if (use)
                for (int m = 0; m < cnt; ++m) {
                    const double4 y = sm[m];
                    acc += green_off<PROB>(P.x - y.x, P.y - y.y, P.z - y.z, hx - y.x, hy - y.y, hz - y.z, r) * y.w;
                }
        }
    }
    if (act) partial[(int64_t)blockIdx.y * n + t] = acc;
}

// Near part: one block per (target, patch) pair, thread c = angle theta_c.
// sigma_j(t_l, theta) = sum_m C_lm cos m theta + S_lm sin m theta, with the
// Fourier coefficients of a chunk of radial nodes formed in LDS from f_j and
// the radial profiles sig[k][l]; points relative to the target as
// (c_j - x) + (cos t - 1) c_j + sin t (cos theta e1_j + sin theta e2_j).
template <int PROB>
__global__ __launch_bounds__(kNearTheta) void k_field_near(
    const double4* __restrict__ pts, const int64_t* __restrict__ pair_t, const int* __restrict__ pair_j,
    const double* __restrict__ frames, const double* __restrict__ coeffs, int K, int M,
    const int* __restrict__ kmode, const int* __restrict__ ptype, const int* __restrict__ t_nr,
    const int64_t* __restrict__ t_roff, const int64_t* __restrict__ t_soff, const double* __restrict__ rad_t_all,
    const double* __restrict__ rad_w_all, const double* __restrict__ sig_all, double* __restrict__ out) {
    __shared__ double F[kNearChunk][2 * kMaxModes];   // [l][m] cos, [l][kMaxModes + m] sin
    __shared__ double fj[136];   // K <= 136 (M <= 15)
    __shared__ double red[kNearTheta / 64];
    const int64_t pr = blockIdx.x;
    const int64_t t = pair_t[pr];
    const int j = pair_j[pr];
    const double4 P = pts[t];
    const double r = P.w;
    const double hs = r > 0.0 ? 1.0 / r : 0.0;
    const double* f = frames + 9 * (int64_t)j;
    // the radial rule and density profiles of patch j's radius
    const int ty = ptype ? ptype[j] : 0;
    const int nr = t_nr[ty];
    const double* rad_t = rad_t_all + t_roff[ty];
    const double* rad_w = rad_w_all + t_roff[ty];
    const double* sig = sig_all + t_soff[ty];
    // target relative to the patch centre (x - c_j and h - c_j)
    const double px = P.x - f[0], py = P.y - f[1], pz = P.z - f[2];
    const double qx = P.x * hs - f[0], qy = P.y * hs - f[1], qz = P.z * hs - f[2];
    for (int k = threadIdx.x; k < K; k += blockDim.x) fj[k] = coeffs[(int64_t)j * K + k];
    const double th = 2.0 * M_PI * threadIdx.x / kNearTheta;
    double cs, sn;
    sincos(th, &sn, &cs);
    // direction in the tangent plane for this angle
    const double ux = cs * f[3] + sn * f[6], uy = cs * f[4] + sn * f[7], uz = cs * f[5] + sn * f[8];
    double cm[kMaxModes], sm[kMaxModes];
    cm[0] = 1.0;
    sm[0] = 0.0;
    for (int m = 1; m <= M; ++m) sincos(m * th, &sm[m], &cm[m]);
    double acc = 0.0;
    for (int l0 = 0; l0 < nr; l0 += kNearChunk) {
        const int cnt = min(kNearChunk, nr - l0);
        __syncthreads();
        if (threadIdx.x < cnt) {
            const int l = l0 + threadIdx.x;
            double c[kMaxModes], s[kMaxModes];
            for (int m = 0; m <= M; ++m) c[m] = s[m] = 0.0;
            for (int k = 0; k < K; ++k) {
                const int mk = kmode[k];
                const double v = fj[k] * sig[(int64_t)k * nr + l];
                if (mk >= 0) c[mk] += v;
                else s[-mk] += v;
            }
            for (int m = 0; m <= M; ++m) {
                F[threadIdx.x][m] = c[m];
                F[threadIdx.x][kMaxModes + m] = s[m];
            }
        }
        __syncthreads();
        for (int li = 0; li < cnt; ++li) {
            const int l = l0 + li;
            double sg = F[li][0];
            for (int m = 1; m <= M; ++m) sg += F[li][m] * cm[m] + F[li][kMaxModes + m] * sm[m];
            const double tl = rad_t[l];
            const double sh = sin(0.5 * tl);
            const double om = -2.0 * sh * sh, st = sin(tl);
            // y - c_j = om c_j + st u
            const double yx = om * f[0] + st * ux, yy = om * f[1] + st * uy, yz = om * f[2] + st * uz;
            acc += rad_w[l] * sg *
                   green_off<PROB>(px - yx, py - yy, pz - yz, qx - yx, qy - yy, qz - yz, r);
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kNearTheta / 64; ++w) s += red[w];
        out[pr] = s * (2.0 * M_PI / kNearTheta);
    }
}

// R_n^m(rho) for every n = m, m+2, ..., M at one rho: R = (-1)^s rho^m
// P_s^(m,0)(1 - 2 rho^2), s = (n - m)/2, by the Jacobi three-term recurrence.
__device__ void zernike_radial_all(int m, int M, double rho, double* R) {
    const double x = 1.0 - 2.0 * rho * rho;
    double rm = 1.0;
    for (int i = 0; i < m; ++i) rm *= rho;
    const double a = m;
    double p0 = 1.0, p1 = 0.5 * (a + (a + 2.0) * x);
    const int smax = (M - m) / 2;
    for (int s = 0; s <= smax; ++s) {
        double ps;
        if (s == 0) {
            ps = p0;
        } else if (s == 1) {
            ps = p1;
        } else {
            const double k2 = 2.0 * s + a;
            const double a1 = 2.0 * s * (s + a) * (k2 - 2.0);
            const double a2 = (k2 - 1.0) * a * a;
            const double a3 = (k2 - 2.0) * (k2 - 1.0) * k2;
            const double a4 = 2.0 * (s + a - 1.0) * (s - 1.0) * k2;
            ps = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
            p0 = p1;
            p1 = ps;
        }
        R[s] = ((s & 1) ? -1.0 : 1.0) * rm * ps;
    }
}

// Self term of a target on the sphere inside patch i: sum_k f_ik Z_k(t/eps_i, theta).
__global__ void k_field_self(int64_t n, const double4* __restrict__ pts, const int* __restrict__ selfp,
                             const double* __restrict__ frames, const double* __restrict__ coeffs, int K, int M,
                             const int* __restrict__ ptype, const double* __restrict__ t_eps,
                             double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int i = selfp[t];
    if (i < 0) {
        out[t] = 0.0;
        return;
    }
    const double4 P = pts[t];
    const double* f = frames + 9 * (int64_t)i;
    const double xc = P.x * f[0] + P.y * f[1] + P.z * f[2];
    const double x1 = P.x * f[3] + P.y * f[4] + P.z * f[5];
    const double x2 = P.x * f[6] + P.y * f[7] + P.z * f[8];
    const double tt = atan2(sqrt(x1 * x1 + x2 * x2), xc);
    const double th = atan2(x2, x1);
    const double eps = t_eps[ptype ? ptype[i] : 0];
    const double rho = fmin(tt / eps, 1.0);
    const double* fi = coeffs + (int64_t)i * K;
    double R[kMaxModes];
    double acc = 0.0;
    // basis order: n ascending, m = -n, -n+2, ..., n; index of (n, m) is
    // n(n+1)/2 + (m + n)/2
    for (int m = 0; m <= M; ++m) {
        zernike_radial_all(m, M, rho, R);
        double sm, cm;
        sincos(m * th, &sm, &cm);
        for (int nn = m; nn <= M; nn += 2) {
            const double rv = R[(nn - m) / 2];
            acc += fi[nn * (nn + 1) / 2 + (m + nn) / 2] * rv * cm;
            if (m > 0) acc += fi[nn * (nn + 1) / 2 + (nn - m) / 2] * rv * sm;
        }
    }
    out[t] = acc;
}

// values[t] = far partial sums + near pair values + self term, then the
// physical field if asked (Is: I_sigma on the device).
__global__ void k_field_combine(int64_t n, int nchunk, const double* __restrict__ partial,
                                const int64_t* __restrict__ nptr, const double* __restrict__ nearv,
                                const double* __restrict__ selfv, const double4* __restrict__ pts, int physical,
                                int problem, const double* __restrict__ Is, double* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double v = selfv[t];
    for (int c = 0; c < nchunk; ++c) v += partial[(int64_t)c * n + t];
    for (int64_t q = nptr[t]; q < nptr[t + 1]; ++q) v += nearv[q];
    if (physical) {
        if (problem == NCE_EXTERIOR) {
            v = 1.0 - v;
        } else {
            const double r = pts[t].w;
            v = (v - 1.0) / (-3.0 * Is[0]) + (1.0 - r * r) / 6.0;
        }
    }
    out[t] = v;
}

}  // namespace
}  // namespace nce

namespace nce_detail {

// Targets (host, n x 3) with their self patch (-1: none; -2: the patch a
// point on the sphere lies on, found here; otherwise a patch of the context's
// order); evaluates the potential (or the physical field) into values_dev.
// coeffs: N x K in the caller's order. Synchronises the stream.
static void field_core(nce_ctx* ctx, const double* coeffs, const std::vector<double>& X, std::vector<int>& selfp,
                       int physical, double* values) {
    const int64_t n = (int64_t)X.size() / 3;
    const int64_t N = ctx->N;
    const int K = ctx->K, M = ctx->tab.M;
    hipStream_t s = ctx->stream;
    const nce::PatchTables& tab = ctx->tab;
    // several radii: patch j of the context has radius type_eps[ptype[j]];
    // its coefficients, frames and tables are in the context's order
    const bool types = ctx->ntype > 1;
    const int ntype = types ? ctx->ntype : 1;
    std::vector<double> teps = types ? ctx->type_eps : std::vector<double>{ctx->eps};
    const int* hptype = types ? ctx->tl.ptype.data() : nullptr;
    auto eps_of = [&](int64_t j) { return teps[hptype ? hptype[j] : 0]; };
    const double eps_max = *std::max_element(teps.begin(), teps.end());
    const double* cf = coeffs;
    if (types) {
        HIPCHK(nce::permute_rows(s, N, K, ctx->d_perm.p, coeffs, ctx->d_xp.p, 0));
        cf = ctx->d_xp.p;
    }
    // patches near each target: centre within arclength 3 eps_j of x/|x|
    // (uniform 3-D cell hash of the centres, cell = chord of 3 eps_max)
    const double cell = 2.0 * std::sin(0.5 * 3.0 * eps_max) * (1.0 + 1e-9);
    auto key = [&](int64_t a, int64_t b, int64_t c) { return (a * 1000003 + b) * 1000033 + c; };
    std::unordered_map<int64_t, std::vector<int>> grid;
    const std::vector<double>& fr = ctx->frames;
    for (int64_t j = 0; j < N; ++j) {
        const double* c = &fr[9 * j];
        grid[key((int64_t)std::floor((c[0] + 1) / cell), (int64_t)std::floor((c[1] + 1) / cell),
                 (int64_t)std::floor((c[2] + 1) / cell))]
            .push_back((int)j);
    }
    std::vector<int64_t> sptr(n + 1, 0), nptr(n + 1, 0);
    std::vector<int> skip, pj;
    std::vector<int64_t> pt;
    std::vector<double> P4(4 * n);
    for (int64_t t = 0; t < n; ++t) {
        const double x = X[3 * t], y = X[3 * t + 1], z = X[3 * t + 2];
        const double r = std::sqrt(x * x + y * y + z * z);
        P4[4 * t] = x;
        P4[4 * t + 1] = y;
        P4[4 * t + 2] = z;
        P4[4 * t + 3] = r;
        std::vector<int> nb;
        int self = selfp[t] == -2 ? -1 : selfp[t];
        double self_ang = 1e300;
        if (r > 0.5 && r < 2.0) {
            const double hx = x / r, hy = y / r, hz = z / r;
            const int64_t ix = (int64_t)std::floor((hx + 1) / cell), iy = (int64_t)std::floor((hy + 1) / cell),
                          iz = (int64_t)std::floor((hz + 1) / cell);
            for (int64_t a = -1; a <= 1; ++a)
                for (int64_t b = -1; b <= 1; ++b)
                    for (int64_t c = -1; c <= 1; ++c) {
                        auto it = grid.find(key(ix + a, iy + b, iz + c));
                        if (it == grid.end()) continue;
                        for (int j : it->second) {
                            const double* cj = &fr[9 * (int64_t)j];
                            const double dt = hx * cj[0] + hy * cj[1] + hz * cj[2];
                            const double cx = hy * cj[2] - hz * cj[1], cy = hz * cj[0] - hx * cj[2],
                                         cz = hx * cj[1] - hy * cj[0];
                            const double ang = std::atan2(std::sqrt(cx * cx + cy * cy + cz * cz), dt);
                            if (ang < 3.0 * eps_of(j)) nb.push_back(j);
                            if (selfp[t] == -2 && ang < self_ang) {
                                self_ang = ang;
                                self = j;
                            }
                        }
                    }
        }
        if (selfp[t] == -2) {
            // on the sphere (to rounding) and within the closed patch of the
            // nearest centre (separation makes that the only candidate)
            const bool on = self >= 0 && std::fabs(r - 1.0) <= 1e-12 && self_ang <= eps_of(self) * (1.0 + 1e-12);
            selfp[t] = on ? self : -1;
        }
        std::sort(nb.begin(), nb.end());
        for (int j : nb) {
            skip.push_back(j);
            if (j != selfp[t]) {
                pt.push_back(t);
                pj.push_back(j);
            }
        }
        if (selfp[t] >= 0 && !std::binary_search(nb.begin(), nb.end(), selfp[t])) {
            // the patch a target lies on is always within 3 eps; kept sorted
            skip.insert(std::upper_bound(skip.begin() + sptr[t], skip.end(), selfp[t]), selfp[t]);
        }
        sptr[t + 1] = (int64_t)skip.size();
        nptr[t + 1] = (int64_t)pj.size();
    }
    const int64_t npair = (int64_t)pj.size();
    DevBuf<double> d_pts, d_partial, d_near, d_self, d_teps, d_Is;
    DevBuf<int64_t> d_sptr, d_nptr, d_pt, d_troff, d_tsigoff;
    DevBuf<int> d_skip, d_pj, d_self_idx, d_kmode, d_tnr;
    DevBuf<double> d_rad_t, d_rad_w, d_sig;
    d_pts.upload(P4, s);
    d_sptr.upload(sptr, s);
    d_nptr.upload(nptr, s);
    if (!skip.empty()) d_skip.upload(skip, s);
    d_self_idx.upload(selfp, s);
    d_teps.upload(teps, s);
    // rho = T f with each radius's base outgoing table (valid at arclength
    // >= 2 eps_j), rows of ldr = the largest base skeleton
    const int ldr = ctx->p;
    if (types) {
        for (int ty = 0; ty < ntype; ++ty) {
            const int64_t a0 = ctx->type_first[ty];
            const int nrow = (int)(ctx->type_first[ty + 1] - a0);
            HIPCHK(nce::gemm_nt<double>(s, nrow, ctx->tabs[ty].p, K, cf + a0 * K, K,
                                        ctx->d_T.p + (int64_t)ctx->type_Toff[ty] * K, K, ctx->d_rho.p + a0 * ldr,
                                        ldr, nullptr, 0));
        }
    } else {
        HIPCHK(nce::gemm_nt<double>(s, (int)N, ldr, K, cf, K, ctx->d_T.p, K, ctx->d_rho.p, ldr, nullptr, 0));
    }
    const int* dptype = types ? ctx->d_ptype.p : nullptr;
    const int* dtsoff = types ? ctx->d_tsoff.p : nullptr;
    const int* dtp = types ? ctx->d_tp.p : nullptr;
    const int ntab = types ? ctx->tl.ntab : 1;
    const int ntb = (int)((n + 255) / 256);
    const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>(N, (2048 + ntb - 1) / ntb));
    const int chunk = (int)((N + nchunk - 1) / nchunk);
    d_partial.alloc((size_t)nchunk * n);
    const dim3 gfar(ntb, nchunk);
    if (tab.problem == NCE_INTERIOR)
        hipLaunchKernelGGL(nce::k_field_far<0>, gfar, dim3(256), 0, s, n, (const double4*)d_pts.p, (int)N, ldr,
                           ctx->d_frames.p, ctx->d_skel_off.p, ctx->d_rho.p, ldr, d_sptr.p, d_skip.p, chunk,
                           d_partial.p, dptype, dtsoff, dtp, ntab);
    else
        hipLaunchKernelGGL(nce::k_field_far<1>, gfar, dim3(256), 0, s, n, (const double4*)d_pts.p, (int)N, ldr,
                           ctx->d_frames.p, ctx->d_skel_off.p, ctx->d_rho.p, ldr, d_sptr.p, d_skip.p, chunk,
                           d_partial.p, dptype, dtsoff, dtp, ntab);
    HIPCHK(hipGetLastError());
    d_near.alloc(std::max<int64_t>(npair, 1));
    if (npair > 0) {
        std::vector<int> zn, zm;
        nce::zernike_modes(M, zn, zm);
        d_kmode.upload(zm, s);
        // each radius's radial rule and density profiles, concatenated
        std::vector<double> rt, rw, sg;
        std::vector<int> tnr;
        std::vector<int64_t> troff, tsoff;
        for (int ty = 0; ty < ntype; ++ty) {
            const nce::PatchTables& tt = types ? ctx->tabs[ty] : tab;
            troff.push_back((int64_t)rt.size());
            tsoff.push_back((int64_t)sg.size());
            tnr.push_back((int)tt.rad_t.size());
            rt.insert(rt.end(), tt.rad_t.begin(), tt.rad_t.end());
            rw.insert(rw.end(), tt.rad_w.begin(), tt.rad_w.end());
            sg.insert(sg.end(), tt.sig.begin(), tt.sig.end());
        }
        d_rad_t.upload(rt, s);
        d_rad_w.upload(rw, s);
        d_sig.upload(sg, s);
        d_tnr.upload(tnr, s);
        d_troff.upload(troff, s);
        d_tsigoff.upload(tsoff, s);
        d_pt.upload(pt, s);
        d_pj.upload(pj, s);
        if (tab.problem == NCE_INTERIOR)
            hipLaunchKernelGGL(nce::k_field_near<0>, dim3((unsigned)npair), dim3(nce::kNearTheta), 0, s,
                               (const double4*)d_pts.p, d_pt.p, d_pj.p, ctx->d_frames.p, cf, K, M, d_kmode.p, dptype,
                               d_tnr.p, d_troff.p, d_tsigoff.p, d_rad_t.p, d_rad_w.p, d_sig.p, d_near.p);
        else
            hipLaunchKernelGGL(nce::k_field_near<1>, dim3((unsigned)npair), dim3(nce::kNearTheta), 0, s,
                               (const double4*)d_pts.p, d_pt.p, d_pj.p, ctx->d_frames.p, cf, K, M, d_kmode.p, dptype,
                               d_tnr.p, d_troff.p, d_tsigoff.p, d_rad_t.p, d_rad_w.p, d_sig.p, d_near.p);
        HIPCHK(hipGetLastError());
    }
    d_self.alloc(n);
    hipLaunchKernelGGL(nce::k_field_self, dim3(ntb), dim3(256), 0, s, n, (const double4*)d_pts.p, d_self_idx.p,
                       ctx->d_frames.p, cf, K, M, dptype, d_teps.p, d_self.p);
    HIPCHK(hipGetLastError());
    const double* Is_dev = ctx->d_scal.p;
    if (physical && tab.problem == NCE_INTERIOR) {
        if (types) {
            // I_sigma: each radius's integral vector over its patches
            for (int ty = 0; ty < ntype; ++ty) {
                const int64_t a0 = ctx->type_first[ty];
                HIPCHK(nce::patch_flux(s, (int)(ctx->type_first[ty + 1] - a0), K, ctx->d_Ityp.p + (size_t)ty * K,
                                       cf + a0 * K, nullptr, ctx->d_partial.p, ctx->d_scal.p + ty));
            }
            std::vector<double> part(ntype);
            HIPCHK(hipMemcpyAsync(part.data(), ctx->d_scal.p, sizeof(double) * ntype, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            double Is = 0.0;
            for (double v : part) Is += v;
            d_Is.upload(std::vector<double>{Is}, s);
            Is_dev = d_Is.p;
        } else {
            HIPCHK(nce::patch_flux(s, (int)N, K, ctx->d_I.p, cf, nullptr, ctx->d_partial.p, ctx->d_scal.p));
        }
    }
    hipLaunchKernelGGL(nce::k_field_combine, dim3(ntb), dim3(256), 0, s, n, nchunk, d_partial.p, d_nptr.p, d_near.p,
                       d_self.p, (const double4*)d_pts.p, physical, tab.problem, Is_dev, values);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace nce_detail

extern "C" {

int nce_field(nce_ctx* ctx, const double* coeffs, const double* points, int64_t n, int physical, double* values) {
    if (!ctx || !coeffs || !points || !values || n < 0) return fail(NCE_EINVAL, "bad argument");
    if (ctx->cfg_first.size() != 2)
        return fail(NCE_ESTATE, "field evaluation needs a single-configuration context");
    if (physical != 0 && physical != 1) return fail(NCE_EINVAL, "physical must be 0 or 1");
    if (n == 0) return NCE_OK;
    return guarded([&]() -> int {
        std::vector<double> X((size_t)3 * n);
        HIPCHK(hipMemcpyAsync(X.data(), points, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        std::vector<int> selfp(n, -2);
        // the representation holds on the problem's side of the sphere; points
        // on the sphere are allowed on either side
        for (int64_t t = 0; t < n; ++t) {
            const double* x = &X[3 * t];
            if (!std::isfinite(x[0]) || !std::isfinite(x[1]) || !std::isfinite(x[2]))
                return fail(NCE_EINVAL, "non-finite point " + std::to_string(t));
            const double r = std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            if (ctx->tab.problem == NCE_INTERIOR ? r > 1.0 + 1e-12 : r < 1.0 - 1e-12)
                return fail(NCE_EINVAL, "point " + std::to_string(t) + " lies outside the domain of the problem");
        }
        field_core(ctx, coeffs, X, selfp, physical, values);
        return NCE_OK;
    });
}

int nce_patch_residual(nce_ctx* ctx, const double* coeffs, const int64_t* patches, int npatch, int n_t,
                       int n_theta, double* residual) {
    if (!ctx || !coeffs || !patches || !residual || npatch < 1 || n_t < 1 || n_theta < 1 || n_t > 64 ||
        n_theta > 256)
        return fail(NCE_EINVAL, "bad argument");
    if (ctx->cfg_first.size() != 2)
        return fail(NCE_ESTATE, "residual evaluation needs a single-configuration context");
    for (int a = 0; a < npatch; ++a)
        if (patches[a] < 0 || patches[a] >= ctx->N) return fail(NCE_EINVAL, "patch index out of range");
    return guarded([&]() -> int {
        // the caller's patch numbers in the context's order, and each one's radius
        std::vector<int64_t> inv;
        if (ctx->ntype > 1) {
            inv.resize(ctx->N);
            for (int64_t a = 0; a < ctx->N; ++a) inv[ctx->perm[a]] = a;
        }
        auto internal = [&](int64_t i) { return inv.empty() ? i : inv[i]; };
        auto eps_of = [&](int64_t a) { return ctx->ntype > 1 ? ctx->type_eps[ctx->tl.ptype[a]] : ctx->eps; };
        std::vector<double> xg, wg;
        nce::gauss_legendre(n_t, xg, wg);
        const int per = n_t * n_theta;
        std::vector<double> X((size_t)3 * per * npatch), W((size_t)per * npatch);
        std::vector<int> selfp((size_t)per * npatch);
        for (int a = 0; a < npatch; ++a) {
            const int64_t ia = internal(patches[a]);
            const double eps = eps_of(ia);
            const double* f = &ctx->frames[9 * ia];
            for (int u = 0; u < n_t; ++u) {
                const double t = 0.5 * eps * (xg[u] + 1.0);
                for (int v = 0; v < n_theta; ++v) {
                    const double th = 2.0 * M_PI * (v + 0.5) / n_theta;
                    const int q = u * n_theta + v;
                    const double ct = std::cos(t), st = std::sin(t), c = std::cos(th), sn = std::sin(th);
                    double* x = &X[3 * ((size_t)a * per + q)];
                    for (int d = 0; d < 3; ++d) x[d] = ct * f[d] + st * (c * f[3 + d] + sn * f[6 + d]);
                    selfp[(size_t)a * per + q] = (int)ia;
                    W[(size_t)a * per + q] = 0.5 * eps * wg[u] * st * (2.0 * M_PI / n_theta);
                }
            }
        }
        DevBuf<double> d_v;
        d_v.alloc((size_t)per * npatch);
        field_core(ctx, coeffs, X, selfp, 0, d_v.p);
        std::vector<double> v((size_t)per * npatch);
        HIPCHK(hipMemcpy(v.data(), d_v.p, sizeof(double) * v.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < npatch; ++a) {
            const double area = 2.0 * M_PI * (1.0 - std::cos(eps_of(internal(patches[a]))));
            double sum = 0.0;
            for (int q = 0; q < per; ++q) {
                const double e = v[(size_t)a * per + q] - 1.0;
                sum += W[(size_t)a * per + q] * e * e;
            }
            residual[a] = std::sqrt(sum) / area;
        }
        return NCE_OK;
    });
}

}  // extern "C"
