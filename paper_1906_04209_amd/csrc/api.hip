// C ABI of the solver (include/nce.h): context, setup, matrix-vector product,
// GMRES and FP64 iterative refinement around an FP32 inner solve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <future>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"

namespace nce_detail {
thread_local std::string g_err;
}
using namespace nce_detail;

namespace nce_detail {

void build_frames(const double* c, int64_t N, std::vector<double>& fr) {
    fr.resize((size_t)N * 9);
    for (int64_t i = 0; i < N; ++i) {
        const double* ci = c + 3 * i;
        double a[3] = {0, 0, 1};
        if (std::fabs(ci[2]) > 1.0 / std::sqrt(2.0)) {
            a[0] = 1;
            a[2] = 0;
        }
        double ad = a[0] * ci[0] + a[1] * ci[1] + a[2] * ci[2];
        double e1[3] = {a[0] - ad * ci[0], a[1] - ad * ci[1], a[2] - ad * ci[2]};
        double nn = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (double& v : e1) v /= nn;
        double e2[3] = {ci[1] * e1[2] - ci[2] * e1[1], ci[2] * e1[0] - ci[0] * e1[2], ci[0] * e1[1] - ci[1] * e1[0]};
        double* f = &fr[(size_t)i * 9];
        for (int k = 0; k < 3; ++k) {
            f[k] = ci[k];
            f[3 + k] = e1[k];
            f[6 + k] = e2[k];
        }
    }
}

void upload_transform_factors(nce_ctx* ctx, hipStream_t s) {
    std::vector<double> trig, rad;
    std::vector<int> mode;
    nce::transform_factors(ctx->tab.M, trig, rad, mode);
    // trig rows zero padded to a multiple of 4 (16-byte reads in the kernel)
    const int nth = 2 * ctx->tab.M + 2, ld = (nth + 3) / 4 * 4, nm = 2 * ctx->tab.M + 1;
    std::vector<double> tp((size_t)nm * ld, 0.0);
    for (int j = 0; j < nm; ++j)
        for (int b = 0; b < nth; ++b) tp[(size_t)j * ld + b] = trig[(size_t)j * nth + b];
    trig.swap(tp);
    ctx->trig_ld = ld;
    ctx->d_Ptrig.upload(trig, s);
    ctx->d_Prad.upload(rad, s);
    ctx->d_Ptrig32.upload(to_f32(trig), s);
    ctx->d_Prad32.upload(to_f32(rad), s);
    ctx->d_Pmode.upload(mode, s);
}

// Every pair of centres closer than 3 eps (arclength) -> NCE_ESEP. Uniform grid
// hash in R^3 with cells of the corresponding chord length.
int check_separation(const double* c, int64_t N, double eps) {
    const double sep = 3.0 * eps;
    const double h = std::max(2.0 * std::sin(std::min(sep, M_PI) / 2.0) * (1.0 + 1e-9), 1e-12);
    const int64_t ncell = (int64_t)std::ceil(2.0 / h) + 2;
    auto key = [&](int64_t x, int64_t y, int64_t z) { return (x * ncell + y) * ncell + z; };
    std::unordered_map<int64_t, std::vector<int64_t>> cells;
    cells.reserve((size_t)N * 2);
    std::vector<int64_t> cx(N), cy(N), cz(N);
    for (int64_t i = 0; i < N; ++i) {
        cx[i] = (int64_t)std::floor((c[3 * i] + 1.0) / h);
        cy[i] = (int64_t)std::floor((c[3 * i + 1] + 1.0) / h);
        cz[i] = (int64_t)std::floor((c[3 * i + 2] + 1.0) / h);
        cells[key(cx[i], cy[i], cz[i])].push_back(i);
    }
    for (int64_t i = 0; i < N; ++i) {
        for (int dx = -1; dx <= 1; ++dx)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dz = -1; dz <= 1; ++dz) {
                    auto it = cells.find(key(cx[i] + dx, cy[i] + dy, cz[i] + dz));
                    if (it == cells.end()) continue;
                    for (int64_t j : it->second) {
                        if (j <= i) continue;
                        const double* a = c + 3 * i;
                        const double* b = c + 3 * j;
                        double cr[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
                        double ang = std::atan2(std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]),
                                                a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
                        if (ang < sep * (1.0 - 1e-12)) {
                            g_err = "patches " + std::to_string(i) + " and " + std::to_string(j) +
                                    " are closer than 3 eps";
                            return NCE_ESEP;
                        }
                    }
                }
    }
    return NCE_OK;
}

void ensure_krylov(nce_ctx* ctx, int nvec) {
    if (ctx->vcap >= nvec) return;
    const size_t n = (size_t)ctx->N * ctx->K;
    ctx->d_V.alloc(n * (size_t)nvec);
    ctx->vcap = nvec;
}

// y = A x for the context's operator in the given precision (enqueued on the
// stream). With ev != nullptr, events ev[0..5] bracket the five steps.
template <class T>
void matvec_t(nce_ctx* ctx, const double* x, double* y, const T* Tm, const T* Pm, const T* noff, const T* soff,
              T* rho, T* U, hipEvent_t* ev, const int* live, int p, int pt) {
    const int N = (int)ctx->N, K = ctx->K, Ks = ctx->Kstar;
    hipStream_t s = ctx->stream;
    auto mark = [&](int k) {
        if (ev) HIPCHK(hipEventRecord(ev[k], s));
    };
    mark(0);
    const T* xin;
    if constexpr (sizeof(T) == 8) {
        xin = reinterpret_cast<const T*>(x);
    } else {
        HIPCHK(nce::cast_d2f(s, (int64_t)N * K, x, ctx->d_x32.p));
        xin = reinterpret_cast<const T*>(ctx->d_x32.p);
    }
    // Step 1: rho_i = T f_i for every patch and every outgoing table in use
    // (one GEMM with the shared, concatenated T; with several radii one GEMM
    // per radius over its range of patches, rows of length ld)
    constexpr bool f64 = sizeof(T) == 8;
    const bool types = ctx->ntype > 1;
    const int ld = types ? (f64 ? ctx->ldr : ctx->ldr32) : pt;
    if (types) {
        const std::vector<int>& Toff = f64 ? ctx->type_Toff : ctx->type_Toff32;
        const std::vector<int>& tp = f64 ? ctx->type_ptot : ctx->type_ptot32;
        for (int ty = 0; ty < ctx->ntype; ++ty) {
            const int64_t a = ctx->type_first[ty];
            const int nr = (int)(ctx->type_first[ty + 1] - a);
            HIPCHK(nce::gemm_nt<T>(s, nr, tp[ty], K, xin + a * K, K, Tm + (int64_t)Toff[ty] * K, K, rho + a * ld, ld,
                                   nullptr, 0));
        }
    } else {
        HIPCHK(nce::gemm_nt<T>(s, N, pt, K, xin, K, Tm, K, rho, pt, nullptr, 0));
    }
    mark(1);
    if (ctx->use_tree) {
        const int ti = sizeof(T) == 8 ? 0 : 1;
        const nce::DeviceTree& dt = (ti == 1 && ctx->has_tree32) ? ctx->dtree32 : ctx->dtree;
        // Step 2: far field onto incoming grids (P2L)
        HIPCHK(nce::tree_far<T>(s, dt, ctx->tab.problem, ctx->d_frames.p, soff, rho, live, ctx->tune_p2l[ti]));
        mark(2);
        // Step 3: leaf neighbours directly at the sampling nodes (writes U)
        HIPCHK(nce::tree_near<T>(s, dt, ctx->tab.problem, ctx->d_frames.p, noff, soff, rho, U, live));
        mark(3);
        // Step 4: interpolation of every ancestor's incoming grid, and Step 5,
        // y = x + P U, in the same kernel's epilogue (U is not written back)
        nce::PApply<T> pa;
        if constexpr (f64) {
            pa.trig = ctx->d_Ptrig.p;
            pa.rad = ctx->d_Prad.p;
        } else {
            pa.trig = ctx->d_Ptrig32.p;
            pa.rad = ctx->d_Prad32.p;
        }
        pa.mode = ctx->d_Pmode.p;
        pa.trig_ld = ctx->trig_ld;
        pa.M = ctx->tab.M;
        pa.K = K;
        pa.x = x;
        pa.y = y;
        HIPCHK(nce::tree_interp<T>(s, dt, ctx->d_frames.p, noff, U, live, ctx->tune_l2t[ti], &pa));
        mark(4);
    } else {
        nce::TypeTabs tt;
        if (types) {
            tt.ptype = ctx->d_ptype.p;
            tt.t_soff = f64 ? ctx->d_tsoff.p : ctx->d_tsoff32.p;
            tt.t_col = f64 ? ctx->d_tcol.p : ctx->d_tcol32.p;
            tt.t_p = f64 ? ctx->d_tp.p : ctx->d_tp32.p;
            tt.ntab = f64 ? ctx->tl.ntab : ctx->tl32.ntab;
            tt.node_stride = 3 * Ks;
        }
        HIPCHK(nce::direct_sum<T>(s, ctx->tab.problem, N, Ks, p, ctx->d_frames.p, noff, soff, rho, U,
                                  ctx->d_logtab.p, tt, ld));
        mark(2);
        mark(3);
        mark(4);
        // Step 5: y = x + P U
        HIPCHK(nce::p_apply<T>(s, N, K, Ks, U, Pm, x, y));
    }
    mark(5);
}

void matvec(nce_ctx* ctx, const double* x, double* y, int precision, hipEvent_t* ev, const int* live) {
    if (ctx->N == 1) {
        if (ev)
            for (int k = 0; k < 6; ++k) HIPCHK(hipEventRecord(ev[k], ctx->stream));
        HIPCHK(hipMemcpyAsync(y, x, sizeof(double) * ctx->K, hipMemcpyDeviceToDevice, ctx->stream));
        return;
    }
    if (precision == NCE_FP64)
        matvec_t<double>(ctx, x, y, ctx->d_T.p, ctx->d_P.p, ctx->d_node_off.p, ctx->d_skel_off.p, ctx->d_rho.p,
                         ctx->d_U.p, ev, live, ctx->p, ctx->ptot);
    else
        matvec_t<float>(ctx, x, y, ctx->d_T32.p, ctx->d_P32.p, ctx->d_node_off32.p, ctx->d_skel_off32.p,
                        ctx->d_rho32.p, ctx->d_U32.p, ev, live, ctx->p32, ctx->ptot32);
}

// total charge of the isolated-patch solution e_0 in a base outgoing table
static double table_chi0(const nce::PatchTables& t) {
    double chi0 = 0.0;
    for (int m = 0; m < t.p; ++m) chi0 += t.T[(size_t)m * t.K];
    return chi0;
}

double coarse_chi0(const nce_ctx* ctx) { return table_chi0(ctx->tab); }

// Several patch radii: every patch's charge chi0 of its own radius, in the
// context's (radius-sorted) patch order; empty for one radius.
std::vector<double> coarse_charges(const nce_ctx* ctx) {
    std::vector<double> chi;
    if (ctx->ntype == 1) return chi;
    chi.resize((size_t)ctx->N);
    for (int t = 0; t < ctx->ntype; ++t)
        std::fill(chi.begin() + ctx->type_first[t], chi.begin() + ctx->type_first[t + 1], table_chi0(ctx->tabs[t]));
    return chi;
}

// Builds the coarse-space deflation of the mixed inner solves and the coarse
// solve (N >= 64).
void ensure_deflation(nce_ctx* ctx) {
    if (ctx->defl || ctx->N < nce::kDeflMinN) return;
    auto d = std::make_unique<nce::Deflation>();
    const std::vector<double> chi = coarse_charges(ctx);
    d->build(ctx->stream, (int)ctx->N, ctx->K, ctx->tab.problem, coarse_chi0(ctx), ctx->frames, ctx->d_frames.p,
             chi.empty() ? nullptr : &chi);
    ctx->d_dtmp.alloc((size_t)ctx->N * ctx->K);
    ctx->defl = std::move(d);
}

// The coarse model's apply through the configuration's tree, O(N log N) in
// place of all pairs: the FP32 far- and near-field kernels on the FP64 tree's
// geometry (its grids, items, direct and interpolation lists), with every
// outgoing table replaced by one point at the patch centre carrying the charge
// chi0_j a_j and one node per patch at its centre; y = a + (near sum +
// interpolated grids). The tree never pairs a patch with itself.
static void install_coarse_tree(nce_ctx* ctx) {
    hipStream_t s = ctx->stream;
    const int64_t N = ctx->N;
    constexpr int kTabs = 64;   // more than any ladder's tables
    ctx->d_ctab_off.upload(std::vector<int>(kTabs, 0), s);
    ctx->d_ctab_p.upload(std::vector<int>(kTabs, 1), s);
    ctx->d_c0.upload(std::vector<float>(3, 0.0f), s);
    ctx->d_cq.alloc((size_t)N);
    ctx->d_cu.alloc((size_t)N);
    ctx->coarse->fast_apply = [ctx, N](hipStream_t st, const double* a, double* y) {
        nce::DeviceTree v = ctx->dtree;   // a view: the tree's own arrays, one-point tables
        v.t_off = ctx->d_ctab_off.p;
        v.t_p = ctx->d_ctab_p.p;
        v.t_col = nullptr;
        v.it_type = nullptr;
        v.ptype = nullptr;
        v.node_stride = 0;
        v.ptot = 1;
        v.p = 1;
        v.Kstar = 1;
        const int problem = ctx->tab.problem;
        const float* c0 = ctx->d_c0.p;
        HIPCHK(ctx->coarse->charges32(st, (int)N, a, ctx->d_cq.p));
        HIPCHK(nce::tree_far<float>(st, v, problem, ctx->d_frames.p, c0, ctx->d_cq.p, nullptr, 4));
        HIPCHK(nce::tree_near<float>(st, v, problem, ctx->d_frames.p, c0, c0, ctx->d_cq.p, ctx->d_cu.p, nullptr));
        HIPCHK(nce::tree_interp<float>(st, v, ctx->d_frames.p, c0, ctx->d_cu.p, nullptr, 2, nullptr));
        HIPCHK(nce::CoarseSolver::finish32(st, (int)N, a, ctx->d_cu.p, y));
    };
}

const double* coarse_amplitudes(nce_ctx* ctx) {
    if (ctx->coarse_iters >= 0) return ctx->d_a.p;
    const double chi0 = coarse_chi0(ctx);
    if (!ctx->coarse) {
        ctx->coarse = std::make_unique<nce::CoarseSolver>((int)ctx->N, ctx->tab.problem, chi0, 80);
        if (ctx->ntype > 1) ctx->coarse->set_charges(ctx->stream, coarse_charges(ctx));
        // the tree's fixed costs (its work items and interpolation blocks are
        // sized for full skeletons) outweigh the N^2 pair sum below about
        // N = 2.5e5 (measured at N = 1e5: 8.3 ms per coarse apply through the
        // tree, 3.8 ms over all pairs); NCE_COARSE_TREE = 1 / 0 forces either
        const char* ev = std::getenv("NCE_COARSE_TREE");
        const bool tree = ev ? std::strcmp(ev, "1") == 0 : ctx->N >= 250000;
        if (tree && ctx->use_tree && ctx->cfg_first.size() == 2) install_coarse_tree(ctx);
    }
    ctx->d_a.alloc((size_t)ctx->N);
    // the deflation's smooth modes are the coarse model's own slow ones: it
    // preconditions this solve as well
    if (ctx->opts.deflation) ensure_deflation(ctx);
    ctx->coarse_iters = ctx->coarse->solve(ctx->stream, (int)ctx->N, ctx->d_frames.p, ctx->opts.tol_coarse, ctx->d_a.p,
                                           ctx->opts.deflation ? ctx->defl.get() : nullptr);
    return ctx->d_a.p;
}

std::vector<float> features_host(nce_ctx* ctx) {
    const double* a = coarse_amplitudes(ctx);
    std::vector<double> ah((size_t)ctx->N);
    HIPCHK(hipMemcpyAsync(ah.data(), a, sizeof(double) * ah.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<float> f;
    nce::patch_features(ctx->frames, ctx->N, ctx->eps, ctx->tab.problem, ah, f);
    return f;
}

namespace {

template <class T>
void autotune_t(nce_ctx* ctx, const T* soff, const T* noff, T* rho, T* U) {
    hipStream_t s = ctx->stream;
    const int ti = sizeof(T) == 8 ? 0 : 1;
    const nce::DeviceTree& d = (ti == 1 && ctx->has_tree32) ? ctx->dtree32 : ctx->dtree;
    // the kernels' cost does not depend on the strengths: start from zeros
    HIPCHK(hipMemsetAsync(rho, 0, sizeof(T) * (size_t)ctx->N * (ti == 0 ? ctx->ptot : ctx->ptot32), s));
    HIPCHK(hipMemsetAsync(U, 0, sizeof(T) * (size_t)ctx->N * ctx->Kstar, s));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    auto best_of = [&](auto&& launch) {
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(e0, s));
            HIPCHK(launch());
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return best;
    };
    try {
        float tbest = 1e30f;
        for (int r : {4, 8, 0, 16}) {
            if (r != 16 && d.max_q > 256 * (r == 4 ? 4 : 8)) continue;
            const float t = best_of([&] {
                return nce::tree_far<T>(s, d, ctx->tab.problem, ctx->d_frames.p, soff, rho, nullptr, r);
            });
            if (t < tbest) {
                tbest = t;
                ctx->tune_p2l[ti] = r;
            }
        }
        tbest = 1e30f;
        for (int npt : {2, 4, 8}) {
            const int threads = npt == 2 ? 256 : (npt == 4 ? 128 : 64);
            if (threads * npt < ctx->Kstar) continue;
            // the fused form the applies run (x = y = the residual buffer as scratch)
            nce::PApply<T> pa;
            if constexpr (sizeof(T) == 8) {
                pa.trig = ctx->d_Ptrig.p;
                pa.rad = ctx->d_Prad.p;
            } else {
                pa.trig = ctx->d_Ptrig32.p;
                pa.rad = ctx->d_Prad32.p;
            }
            pa.mode = ctx->d_Pmode.p;
            pa.trig_ld = ctx->trig_ld;
            pa.M = ctx->tab.M;
            pa.K = ctx->K;
            pa.x = ctx->d_r.p;
            pa.y = ctx->d_r.p;
            const float t =
                best_of([&] { return nce::tree_interp<T>(s, d, ctx->d_frames.p, noff, U, nullptr, npt, &pa); });
            if (t < tbest) {
                tbest = t;
                ctx->tune_l2t[ti] = npt;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
}

}  // namespace

void autotune(nce_ctx* ctx, int precision) {
    if (!ctx->use_tree) return;
    if ((precision == NCE_FP64 || !ctx->has_tree32) ? ctx->dtree.ngrid == 0 : ctx->dtree32.ngrid == 0) return;
    if (precision == NCE_FP64)
        autotune_t<double>(ctx, ctx->d_skel_off.p, ctx->d_node_off.p, ctx->d_rho.p, ctx->d_U.p);
    else
        autotune_t<float>(ctx, ctx->d_skel_off32.p, ctx->d_node_off32.p, ctx->d_rho32.p, ctx->d_U32.p);
}

double dev_dot(nce_ctx* ctx, int64_t n, const double* a, const double* b) {
    HIPCHK(nce::dots(ctx->stream, n, 1, a, n, b, ctx->d_partial.p, ctx->d_scal.p));
    double v = 0;
    HIPCHK(hipMemcpyAsync(&v, ctx->d_scal.p, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return v;
}

// GMRES (unrestarted, CGS2 Arnoldi on the device, Givens on the host) for
// A x = rhs with x = 0 initially; adds the solution into x. Stops when the
// residual estimate is <= tol * ||rhs||. Returns the number of matvecs.
int gmres(nce_ctx* ctx, const double* rhs, double* x, double tol, int maxit, int precision, bool& converged,
          double& est_rel) {
    const int64_t n = ctx->N * (int64_t)ctx->K;
    hipStream_t s = ctx->stream;
    ensure_krylov(ctx, maxit + 1);
    double* V = ctx->d_V.p;
    const bool defl = precision == NCE_MIXED && ctx->opts.deflation && ctx->defl;
    const double bnorm = std::sqrt(dev_dot(ctx, n, rhs, rhs));
    converged = false;
    est_rel = 1.0;
    if (bnorm == 0.0) {
        converged = true;
        est_rel = 0.0;
        return 0;
    }
    HIPCHK(nce::scale_copy(s, n, 1.0 / bnorm, rhs, V));
    std::vector<double> H((size_t)(maxit + 1) * maxit, 0.0), cs(maxit), sn(maxit), g(maxit + 1, 0.0);
    std::vector<double> h(maxit + 1), h2(maxit + 1);
    g[0] = bnorm;
    int k = 0, used = 0;
    for (k = 0; k < maxit; ++k) {
        double* w = V + (int64_t)(k + 1) * n;
        if (defl) {
            // right preconditioning: w = A M^{-1} v_k
            HIPCHK(ctx->defl->apply(s, V + (int64_t)k * n, ctx->d_dtmp.p));
            matvec(ctx, ctx->d_dtmp.p, w, precision);
        } else {
            matvec(ctx, V + (int64_t)k * n, w, precision);
        }
        used++;
        // classical Gram-Schmidt on FP64 vectors: twice for the FP64 solves;
        // once for the FP32 inner solves of the mixed form, whose 1e-5 target
        // is far above the orthogonality lost in one FP64 pass
        const int passes = precision == NCE_MIXED ? 1 : 2;
        std::fill(h2.begin(), h2.end(), 0.0);
        for (int pass = 0; pass < passes; ++pass) {
            HIPCHK(nce::dots(s, n, k + 1, V, n, w, ctx->d_partial.p, ctx->d_h.p));
            HIPCHK(nce::axpys(s, n, k + 1, V, n, ctx->d_h.p, w));
            HIPCHK(hipMemcpyAsync(pass == 0 ? h.data() : h2.data(), ctx->d_h.p, sizeof(double) * (k + 1),
                                  hipMemcpyDeviceToHost, s));
        }
        HIPCHK(nce::dots(s, n, 1, w, n, w, ctx->d_partial.p, ctx->d_scal.p));
        double hk1sq = 0;
        HIPCHK(hipMemcpyAsync(&hk1sq, ctx->d_scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double hk1 = std::sqrt(hk1sq);
        if (!std::isfinite(hk1)) throw std::runtime_error("non-finite Arnoldi norm");
        for (int j = 0; j <= k; ++j) H[(size_t)j * maxit + k] = h[j] + h2[j];
        H[(size_t)(k + 1) * maxit + k] = hk1;
        for (int j = 0; j < k; ++j) {
            double a = H[(size_t)j * maxit + k], b = H[(size_t)(j + 1) * maxit + k];
            H[(size_t)j * maxit + k] = cs[j] * a + sn[j] * b;
            H[(size_t)(j + 1) * maxit + k] = -sn[j] * a + cs[j] * b;
        }
        double a = H[(size_t)k * maxit + k], b = H[(size_t)(k + 1) * maxit + k];
        double den = std::hypot(a, b);
        cs[k] = a / den;
        sn[k] = b / den;
        H[(size_t)k * maxit + k] = den;
        H[(size_t)(k + 1) * maxit + k] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        est_rel = std::fabs(g[k + 1]) / bnorm;
        const bool happy = hk1 <= 1e-14 * bnorm;
        if (est_rel <= tol || happy) {
            converged = true;
            k++;
            break;
        }
        HIPCHK(nce::scale_copy(s, n, 1.0 / hk1, w, w));
    }
    const int m = std::min(k, maxit);
    std::vector<double> y(m);
    for (int i = m - 1; i >= 0; --i) {
        double acc = g[i];
        for (int j = i + 1; j < m; ++j) acc -= H[(size_t)i * maxit + j] * y[j];
        y[i] = acc / H[(size_t)i * maxit + i];
    }
    HIPCHK(hipMemcpyAsync(ctx->d_h.p, y.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    if (defl) {
        // x += M^{-1} (V y)
        HIPCHK(nce::fill(s, n, 0.0, ctx->d_dtmp.p));
        HIPCHK(nce::combine(s, n, m, V, n, ctx->d_h.p, ctx->d_dtmp.p));
        HIPCHK(ctx->defl->apply(s, ctx->d_dtmp.p, ctx->d_dtmp.p));
        HIPCHK(nce::axpby(s, n, 1.0, ctx->d_dtmp.p, 1.0, x));
    } else {
        HIPCHK(nce::combine(s, n, m, V, n, ctx->d_h.p, x));
    }
    return used;
}

// r = b - A x in FP64; returns ||r|| / ||b||.
double residual(nce_ctx* ctx, const double* b, const double* x, double* r) {
    const int64_t n = ctx->N * (int64_t)ctx->K;
    matvec(ctx, x, r, NCE_FP64);
    HIPCHK(nce::axpby(ctx->stream, n, 1.0, b, -1.0, r));
    const double rn = std::sqrt(dev_dot(ctx, n, r, r));
    const double bn = std::sqrt(dev_dot(ctx, n, b, b));
    return rn / bn;
}

int solve(nce_ctx* ctx, double* coeffs, double* flux, double* Is_out, nce_info* info) {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t N = ctx->N, n = N * (int64_t)ctx->K;
    hipStream_t s = ctx->stream;
    nce_info inf{};
    // coarse-space deflation of the inner solves, once per context (inside the timed solve)
    if (ctx->opts.precision == NCE_MIXED && ctx->opts.deflation) ensure_deflation(ctx);
    // b = P 1 = e_0 on every patch
    if (ctx->d_b.n < (size_t)n) ctx->d_b.alloc((size_t)n);
    HIPCHK(nce::unit_rhs(s, N, ctx->K, ctx->d_b.p));
    double* x = ctx->d_x.p;
    HIPCHK(nce::fill(s, n, 0.0, x));
    const double tol = ctx->opts.tol_gmres;
    const int maxit = ctx->opts.max_iter;
    bool conv = false;
    double est = 1.0;
    // r = residual of the current x, rel = ||r|| / ||b||
    HIPCHK(hipMemcpyAsync(ctx->d_r.p, ctx->d_b.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
    double rel = 1.0;
    if ((ctx->warm_coarse || ctx->warm) && N > 1) {
        // initial guess from the monopole (coarse) solve a, refined per patch by
        // the network's shape factors m_i: x0_i = a_i m_i (a_i e_0 without one)
        const double* a = coarse_amplitudes(ctx);
        const float* m32 = nullptr;
        if (ctx->warm) {
            if (!ctx->d_feat.p) ctx->d_feat.upload(features_host(ctx), s);
            m32 = ctx->warm->forward(s, ctx->d_feat.p, N);
        }
        HIPCHK(nce::rows_scale(s, N, ctx->K, a, m32, x));
        if (ctx->opts.precision == NCE_MIXED) {
            // r0 with the FP32 apply first: when the guess is good enough for one
            // refinement step to reach the tolerance (r0 <= tol / 1e-5, the FP32
            // solve's floor) r0 is recomputed in FP64; otherwise the refinement
            // starts from this estimate and verifies in FP64 after its first step
            matvec(ctx, x, ctx->d_r.p, NCE_MIXED);
            HIPCHK(nce::axpby(s, n, 1.0, ctx->d_b.p, -1.0, ctx->d_r.p));
            rel = std::sqrt(dev_dot(ctx, n, ctx->d_r.p, ctx->d_r.p) / dev_dot(ctx, n, ctx->d_b.p, ctx->d_b.p));
            inf.iters_fp32++;
            if (rel <= tol / 1e-5) {
                rel = residual(ctx, ctx->d_b.p, x, ctx->d_r.p);
                inf.iters_fp64++;
            }
        } else {
            // r = b - A x0 in FP64 (one apply)
            rel = residual(ctx, ctx->d_b.p, x, ctx->d_r.p);
            inf.iters_fp64++;
        }
        inf.rel_residual_x0 = rel;
        if (!(rel < 0.99)) {
            // no gain: plain start from zero
            inf.used_fallback = 1;
            HIPCHK(nce::fill(s, n, 0.0, x));
            HIPCHK(hipMemcpyAsync(ctx->d_r.p, ctx->d_b.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
            rel = 1.0;
        }
    }
    if (N == 1) {
        // one patch: the system matrix is the identity (no scattering), x = b
        HIPCHK(hipMemcpyAsync(x, ctx->d_b.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        conv = true;
        inf.rel_residual = 0.0;
        inf.rel_residual_x0 = 1.0;
    } else if (ctx->opts.precision == NCE_FP64) {
        if (!(ctx->warm || ctx->warm_coarse)) inf.rel_residual_x0 = 1.0;
        // GMRES on A d = r with ||r - A d|| <= tol ||b||; x += d
        inf.iters_fp64 += gmres(ctx, ctx->d_r.p, x, tol / rel, maxit, NCE_FP64, conv, est);
        inf.rel_residual = residual(ctx, ctx->d_b.p, x, ctx->d_r.p);
        inf.outer = 1;
    } else {
        // FP64 iterative refinement: r = b - A64 x; A32 d = r by GMRES; x += d.
        if (!(ctx->warm || ctx->warm_coarse)) inf.rel_residual_x0 = rel;
        const int max_outer = 12;
        conv = false;
        for (int outer = 0; outer < max_outer; ++outer) {
            const double inner_tol = std::max(1e-5, 0.5 * tol / rel);
            bool c2;
            double e2;
            inf.iters_fp32 += gmres(ctx, ctx->d_r.p, x, inner_tol, maxit, NCE_MIXED, c2, e2);
            inf.outer++;
            const double prev = rel;
            rel = residual(ctx, ctx->d_b.p, x, ctx->d_r.p);
            inf.iters_fp64 += 1;
            if (rel <= tol) {
                conv = true;
                break;
            }
            if (!(rel < 0.5 * prev)) {
                // refinement stalled: finish with FP64 GMRES on the residual
                inf.used_fallback = 1;
                bool c3;
                double e3;
                inf.iters_fp64 += gmres(ctx, ctx->d_r.p, x, tol / rel, maxit, NCE_FP64, c3, e3);
                rel = residual(ctx, ctx->d_b.p, x, ctx->d_r.p);
                inf.iters_fp64 += 1;
                conv = rel <= tol * 1.0001 || c3;
                break;
            }
        }
        inf.rel_residual = rel;
    }
    double Is = 0;
    if (ctx->ntype > 1) {
        // each radius's integral vector over its patches; outputs in the caller's order
        double* fl = flux ? ctx->d_fluxp.p : nullptr;
        for (int ty = 0; ty < ctx->ntype; ++ty) {
            const int64_t a = ctx->type_first[ty];
            HIPCHK(nce::patch_flux(s, (int)(ctx->type_first[ty + 1] - a), ctx->K, ctx->d_Ityp.p + (size_t)ty * ctx->K,
                                   x + a * ctx->K, fl ? fl + a : nullptr, ctx->d_partial.p, ctx->d_scal.p + ty));
        }
        double part[8];
        HIPCHK(hipMemcpyAsync(part, ctx->d_scal.p, sizeof(double) * ctx->ntype, hipMemcpyDeviceToHost, s));
        if (coeffs) HIPCHK(nce::permute_rows(s, N, ctx->K, ctx->d_perm.p, x, coeffs, 1));
        if (flux) HIPCHK(nce::permute_rows(s, N, 1, ctx->d_perm.p, fl, flux, 1));
        HIPCHK(hipStreamSynchronize(s));
        for (int ty = 0; ty < ctx->ntype; ++ty) Is += part[ty];
    } else {
        HIPCHK(nce::patch_flux(s, (int)N, ctx->K, ctx->d_I.p, x, flux, ctx->d_partial.p, ctx->d_scal.p));
        HIPCHK(hipMemcpyAsync(&Is, ctx->d_scal.p, sizeof(double), hipMemcpyDeviceToHost, s));
        if (coeffs) HIPCHK(hipMemcpyAsync(coeffs, x, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    *Is_out = Is;
    inf.t_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return (conv && inf.rel_residual <= tol * 1.0001) ? NCE_OK : NCE_NOTCONVERGED;
}


int validate_opts(const nce_opts& o, double eps) {
    if (!(eps > 0.0 && eps <= M_PI / 3.0)) return fail(NCE_EINVAL, "eps must lie in (0, pi/3]");
    if (o.M < 0 || o.M > 15)
        return fail(NCE_EINVAL, "M must lie in [0, 15] (at most 2 (M+1)^2 = 512 Zernike sampling nodes per patch)");
    if (o.problem != NCE_INTERIOR && o.problem != NCE_EXTERIOR) return fail(NCE_EINVAL, "bad problem");
    if (!(o.tol_id > 0 && o.tol_id < 1e-3)) return fail(NCE_EINVAL, "tol_id must lie in (0, 1e-3)");
    if (!(o.tol_grid > 0 && o.tol_grid < 1e-2)) return fail(NCE_EINVAL, "tol_grid must lie in (0, 1e-2)");
    if (!(o.tol_grid_fp32 == 0.0 || (o.tol_grid_fp32 > 0 && o.tol_grid_fp32 < 1e-2)))
        return fail(NCE_EINVAL, "tol_grid_fp32 must be 0 or lie in (0, 1e-2)");
    if (!(o.tol_id_fp32 == 0.0 || (o.tol_id_fp32 > 0 && o.tol_id_fp32 < 1e-3)))
        return fail(NCE_EINVAL, "tol_id_fp32 must be 0 or lie in (0, 1e-3)");
    if (!(o.tol_coarse > 0 && o.tol_coarse < 0.1)) return fail(NCE_EINVAL, "tol_coarse must lie in (0, 0.1)");
    if (o.deflation != 0 && o.deflation != 1) return fail(NCE_EINVAL, "deflation must be 0 or 1");
    if (!(o.tol_gmres > 0 && o.tol_gmres < 1)) return fail(NCE_EINVAL, "tol_gmres must lie in (0, 1)");
    if (o.max_iter < 1 || o.max_iter > 2000) return fail(NCE_EINVAL, "max_iter must lie in [1, 2000]");
    if (o.precision != NCE_FP64 && o.precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    if (o.far_field != NCE_FAR_AUTO && o.far_field != NCE_FAR_DIRECT && o.far_field != NCE_FAR_TREE)
        return fail(NCE_EINVAL, "bad far_field");
    return NCE_OK;
}

int validate_centers(const double* centers, const std::vector<int64_t>& cfg_first, double eps) {
    const int64_t N = cfg_first.back();
    for (int64_t i = 0; i < N; ++i) {
        const double* c = centers + 3 * i;
        if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2]))
            return fail(NCE_EINVAL, "non-finite centre " + std::to_string(i));
        double nn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (std::fabs(nn - 1.0) > 1e-12) return fail(NCE_EINVAL, "centre " + std::to_string(i) + " is not a unit vector");
    }
    for (size_t c = 0; c + 1 < cfg_first.size(); ++c) {
        const int rc = check_separation(centers + 3 * cfg_first[c], cfg_first[c + 1] - cfg_first[c], eps);
        if (rc != NCE_OK) {
            if (cfg_first.size() > 2) g_err = "configuration " + std::to_string(c) + ": " + g_err;
            return rc;
        }
    }
    return NCE_OK;
}

void init_ctx(nce_ctx* ctx, const double* centers, const std::vector<int64_t>& cfg_first, double eps,
              const nce_opts& o, bool forest) {
    const int64_t N = cfg_first.back();
    ctx->opts = o;
    ctx->N = N;
    ctx->eps = eps;
    ctx->cfg_first = cfg_first;
    if (o.stream) {
        ctx->stream = (hipStream_t)o.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    std::string dir;
    if (o.cache_dir) dir = o.cache_dir;
    else if (const char* e = std::getenv("NCE_CACHE")) dir = e;
    // tables not in the cache are built with their modal solves and IDs on the
    // GPU (NCE_HOST_PRECOMPUTE=1: all on the host)
    std::unique_ptr<nce::PrecomputeDevice> pdev;
    {
        const char* hp = std::getenv("NCE_HOST_PRECOMPUTE");
        if (!(hp && hp[0] == '1')) pdev = nce::make_gpu_precompute(ctx->stream);
    }
    if (!nce::load_tables(dir, o.problem, eps, o.M, o.tol_id, ctx->tab)) {
        ctx->tab = nce::build_tables(o.problem, eps, o.M, o.tol_id, 0, pdev.get());
        nce::save_tables(dir, ctx->tab);
    }
    ctx->K = ctx->tab.K;
    ctx->Kstar = ctx->tab.Kstar;
    ctx->p = ctx->tab.p;
    // the FP32 applies may use a coarser outgoing representation
    const double tid32 = o.tol_id_fp32 > 0 ? o.tol_id_fp32 : o.tol_id;
    ctx->has_tab32 = tid32 != o.tol_id;
    if (ctx->has_tab32 && !nce::load_tables(dir, o.problem, eps, o.M, tid32, ctx->tab32)) {
        ctx->tab32 = nce::build_tables(o.problem, eps, o.M, tid32, 0, pdev.get());
        nce::save_tables(dir, ctx->tab32);
    }
    const nce::PatchTables& t32 = ctx->has_tab32 ? ctx->tab32 : ctx->tab;
    ctx->p32 = t32.p;
    build_frames(centers, N, ctx->frames);
    hipStream_t s = ctx->stream;
    const size_t n = (size_t)N * ctx->K;
    // far field of a single configuration: the tree or the direct all-pairs sum
    // as opts.far_field says, or (automatic) whichever has the smaller operation
    // count (one interpolation FMA is priced at a quarter of a Green's function
    // pair, from the FP32 instruction mixes of the two kernels)
    if (forest) {
        ctx->use_tree = true;
    } else if (N < 2 || o.far_field == NCE_FAR_DIRECT) {
        ctx->use_tree = false;
    } else {
        nce::build_tree(ctx->frames, N, eps, ctx->tab, o.tol_grid, ctx->tree);
        const double direct = (double)N * (double)(N - 1) * ctx->tab.Kstar * (double)ctx->tab.p;
        const double viatree = ctx->tree.pairs_far + ctx->tree.pairs_near + 0.25 * ctx->tree.interp_fma;
        ctx->use_tree = o.far_field == NCE_FAR_TREE || viatree < direct;
        if (!ctx->use_tree) ctx->tree = nce::Tree();
    }
    // outgoing tables: the base representation, then (tree only) the
    // recompressions for far targets, concatenated row-wise
    std::vector<double> Tall(ctx->tab.T), soff(ctx->tab.skel_off);
    ctx->tab_off = {0};
    ctx->tab_p = {ctx->p};
    if (ctx->use_tree) {
        for (const auto& ft : ctx->tab.far) {
            ctx->tab_off.push_back(ctx->tab_off.back() + ctx->tab_p.back());
            ctx->tab_p.push_back(ft.p);
            Tall.insert(Tall.end(), ft.T.begin(), ft.T.end());
            soff.insert(soff.end(), ft.skel_off.begin(), ft.skel_off.end());
        }
    }
    ctx->ptot = ctx->tab_off.back() + ctx->tab_p.back();
    std::vector<double> Tall32(t32.T), soff32(t32.skel_off);
    ctx->tab_off32 = {0};
    ctx->tab_p32 = {ctx->p32};
    if (ctx->use_tree) {
        for (const auto& ft : t32.far) {
            ctx->tab_off32.push_back(ctx->tab_off32.back() + ctx->tab_p32.back());
            ctx->tab_p32.push_back(ft.p);
            Tall32.insert(Tall32.end(), ft.T.begin(), ft.T.end());
            soff32.insert(soff32.end(), ft.skel_off.begin(), ft.skel_off.end());
        }
    }
    ctx->ptot32 = ctx->tab_off32.back() + ctx->tab_p32.back();
    ctx->d_frames.upload(ctx->frames, s);
    ctx->d_T.upload(Tall, s);
    ctx->d_P.upload(ctx->tab.P, s);
    ctx->d_I.upload(ctx->tab.I, s);
    ctx->d_node_off.upload(ctx->tab.node_off, s);
    ctx->d_skel_off.upload(soff, s);
    ctx->d_T32.upload(to_f32(Tall32), s);
    ctx->d_P32.upload(to_f32(ctx->tab.P), s);
    upload_transform_factors(ctx, s);
    ctx->d_node_off32.upload(to_f32(ctx->tab.node_off), s);
    ctx->d_skel_off32.upload(to_f32(soff32), s);
    {
        std::vector<nce::LogEntry> lt(nce::kLogTab);
        nce::build_log_table(lt.data());
        ctx->d_logtab.upload(lt, s);
    }
    ctx->d_rho.alloc((size_t)N * ctx->ptot);
    ctx->d_U.alloc((size_t)N * ctx->Kstar);
    ctx->d_rho32.alloc((size_t)N * ctx->ptot32);
    ctx->d_U32.alloc((size_t)N * ctx->Kstar);
    ctx->d_x32.alloc(n);
    ctx->d_b.alloc(n);
    ctx->d_r.alloc(n);
    ctx->d_x.alloc(n);
    ctx->d_h.alloc((size_t)o.max_iter + 8);
    ctx->d_partial.alloc((size_t)nce::kReduceBlocks * ((size_t)o.max_iter + 8));
    ctx->d_scal.alloc(8);
    const int ncfg = (int)cfg_first.size() - 1;
    ctx->cfg_tree.assign(ncfg, ctx->use_tree ? 1 : 0);
    const double tol32 = o.tol_grid_fp32 > 0 ? o.tol_grid_fp32 : o.tol_grid;
    ctx->has_tree32 = ctx->use_tree && (tol32 != o.tol_grid || ctx->has_tab32);
    if (forest) {
        nce::start_forest(ctx->tree);
        if (ctx->has_tree32) nce::start_forest(ctx->tree32);
        for (int c = 0; c < ncfg; ++c) {
            const int64_t f0 = cfg_first[c], nc = cfg_first[c + 1] - f0;
            bool tree = nc > 1 && o.far_field != NCE_FAR_DIRECT;
            nce::Tree t;
            std::vector<double> fr;
            if (tree) {
                fr.assign(ctx->frames.begin() + 9 * f0, ctx->frames.begin() + 9 * (f0 + nc));
                nce::build_tree(fr, nc, eps, ctx->tab, o.tol_grid, t);
                if (o.far_field == NCE_FAR_AUTO) {
                    // operation counts: one interpolation FMA costs about a quarter of a
                    // Green's function pair (FP32 instruction mix of the two kernels)
                    const double direct = (double)nc * (double)(nc - 1) * ctx->Kstar * (double)ctx->p;
                    const double viatree = t.pairs_far + t.pairs_near + 0.25 * t.interp_fma;
                    tree = viatree < direct;
                }
            }
            ctx->cfg_tree[c] = tree ? 1 : 0;
            if (tree) nce::append_tree(ctx->tree, t, f0);
            else nce::append_direct(ctx->tree, f0, nc, ctx->Kstar, ctx->p);
            if (ctx->has_tree32) {
                if (tree) {
                    nce::Tree tr32;
                    nce::build_tree(fr, nc, eps, t32, tol32, tr32, false);
                    nce::append_tree(ctx->tree32, tr32, f0);
                } else {
                    nce::append_direct(ctx->tree32, f0, nc, ctx->Kstar, ctx->p32);
                }
            }
        }
    } else if (ctx->has_tree32) {
        nce::build_tree(ctx->frames, N, eps, t32, tol32, ctx->tree32, false);
    }
    if (ctx->use_tree) nce::upload_tree(ctx->tree, ctx->Kstar, ctx->p, ctx->tab_off, ctx->tab_p, s, ctx->dtree);
    if (ctx->has_tree32)
        nce::upload_tree(ctx->tree32, ctx->Kstar, ctx->p32, ctx->tab_off32, ctx->tab_p32, s, ctx->dtree32);
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace nce_detail

extern "C" {

void nce_default_opts(nce_opts* o) {
    if (!o) return;
    o->problem = NCE_INTERIOR;
    o->M = 15;
    o->tol_id = 1e-11;
    o->tol_grid = 1e-8;
    o->tol_gmres = 1e-10;
    o->max_iter = 100;
    o->precision = NCE_FP64;
    o->far_field = NCE_FAR_AUTO;
    o->stream = nullptr;
    o->cache_dir = nullptr;
    o->tol_grid_fp32 = 3e-4;
    o->tol_id_fp32 = 1e-5;
    o->tol_coarse = 1e-5;
    o->deflation = 1;
}

int nce_setup(const double* centers, int64_t N, double eps, const nce_opts* opts_in, nce_ctx** out) {
    g_err.clear();
    if (!out) return fail(NCE_EINVAL, "out is NULL");
    *out = nullptr;
    nce_opts o;
    nce_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (!centers || N < 1) return fail(NCE_EINVAL, "need N >= 1 centres");
    int rc = validate_opts(o, eps);
    if (rc != NCE_OK) return rc;
    const std::vector<int64_t> cfg_first{0, N};
    rc = validate_centers(centers, cfg_first, eps);
    if (rc != NCE_OK) return rc;
    return guarded([&]() -> int {
        auto* ctx = new nce_ctx();
        std::unique_ptr<nce_ctx, void (*)(nce_ctx*)> guard(ctx, nce_destroy);
        init_ctx(ctx, centers, cfg_first, eps, o, false);
        *out = guard.release();
        return NCE_OK;
    });
}

void nce_destroy(nce_ctx* ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    nce::free_tree(ctx->dtree);
    nce::free_tree(ctx->dtree32);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

int nce_dims(const nce_ctx* ctx, int* K, int* Kstar, int* p, int* levels) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (K) *K = ctx->K;
    if (Kstar) *Kstar = ctx->Kstar;
    if (p) *p = ctx->p;
    if (levels) *levels = ctx->use_tree ? ctx->tree.nlevels : 0;
    return NCE_OK;
}

int nce_frames(const nce_ctx* ctx, double* fr) {
    if (!ctx || !fr) return fail(NCE_EINVAL, "NULL argument");
    if (ctx->ntype > 1) {
        for (int64_t a = 0; a < ctx->N; ++a)
            std::memcpy(fr + 9 * ctx->perm[a], ctx->frames.data() + 9 * a, sizeof(double) * 9);
    } else {
        std::memcpy(fr, ctx->frames.data(), sizeof(double) * ctx->frames.size());
    }
    return NCE_OK;
}

int nce_work(const nce_ctx* ctx, int precision, double* far, double* near, double* interp) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    double f = 0, nr = 0, it = 0;
    if (ctx->use_tree) {
        const nce::Tree& t = (precision == NCE_MIXED && ctx->has_tree32) ? ctx->tree32 : ctx->tree;
        f = t.pairs_far;
        nr = t.pairs_near;
        it = t.interp_fma;
    } else {
        f = (double)ctx->N * (double)(ctx->N - 1) * ctx->Kstar * (double)(precision == NCE_MIXED ? ctx->p32 : ctx->p);
    }
    if (far) *far = f;
    if (near) *near = nr;
    if (interp) *interp = it;
    return NCE_OK;
}

int nce_matvec(nce_ctx* ctx, const double* x, double* y, int precision) {
    if (!ctx || !x || !y) return fail(NCE_EINVAL, "NULL argument");
    if (x == y) return fail(NCE_EINVAL, "x and y may not alias");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        if (ctx->ntype > 1) {
            // the context holds its patches sorted by radius
            HIPCHK(nce::permute_rows(ctx->stream, ctx->N, ctx->K, ctx->d_perm.p, x, ctx->d_xp.p, 0));
            matvec(ctx, ctx->d_xp.p, ctx->d_yp.p, precision);
            HIPCHK(nce::permute_rows(ctx->stream, ctx->N, ctx->K, ctx->d_perm.p, ctx->d_yp.p, y, 1));
        } else {
            matvec(ctx, x, y, precision);
        }
        return NCE_OK;
    });
}

int nce_matvec_profile(nce_ctx* ctx, const double* x, double* y, int precision, double* step_ms) {
    if (!ctx || !x || !y || !step_ms) return fail(NCE_EINVAL, "NULL argument");
    if (x == y) return fail(NCE_EINVAL, "x and y may not alias");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        hipEvent_t ev[6] = {};
        for (auto& e : ev) HIPCHK(hipEventCreate(&e));
        try {
            if (ctx->ntype > 1) {
                HIPCHK(nce::permute_rows(ctx->stream, ctx->N, ctx->K, ctx->d_perm.p, x, ctx->d_xp.p, 0));
                matvec(ctx, ctx->d_xp.p, ctx->d_yp.p, precision, ev);
                HIPCHK(nce::permute_rows(ctx->stream, ctx->N, ctx->K, ctx->d_perm.p, ctx->d_yp.p, y, 1));
            } else {
                matvec(ctx, x, y, precision, ev);
            }
            HIPCHK(hipEventSynchronize(ev[5]));
            for (int k = 0; k < 5; ++k) {
                float ms = 0;
                HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
                step_ms[k] = ms;
            }
        } catch (...) {
            for (auto& e : ev) (void)hipEventDestroy(e);
            throw;
        }
        for (auto& e : ev) (void)hipEventDestroy(e);
        return NCE_OK;
    });
}

int nce_autotune(nce_ctx* ctx, int precision, int* choice) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        autotune(ctx, precision);
        const int ti = precision == NCE_FP64 ? 0 : 1;
        if (choice) {
            choice[0] = ctx->tune_p2l[ti];
            choice[1] = ctx->tune_l2t[ti];
        }
        return NCE_OK;
    });
}

int nce_set_shapes(nce_ctx* ctx, int precision, int p2l_shape, int l2t_npt) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    if (p2l_shape != 0 && p2l_shape != 4 && p2l_shape != 8 && p2l_shape != 16)
        return fail(NCE_EINVAL, "P2L shape must be 0, 4, 8 or 16");
    if (l2t_npt != 2 && l2t_npt != 4 && l2t_npt != 8) return fail(NCE_EINVAL, "interpolation nodes per thread: 2, 4 or 8");
    const int ti = precision == NCE_FP64 ? 0 : 1;
    if (ctx->use_tree) {
        const nce::DeviceTree& d = (ti == 1 && ctx->has_tree32) ? ctx->dtree32 : ctx->dtree;
        if (p2l_shape != 16 && d.max_q > 256 * (p2l_shape == 4 ? 4 : 8))
            return fail(NCE_EINVAL, "a grid of this tree is too large for that P2L shape");
    }
    ctx->tune_p2l[ti] = p2l_shape;
    ctx->tune_l2t[ti] = l2t_npt;
    return NCE_OK;
}

int nce_set_solver(nce_ctx* ctx, double tol, int max_iter, int precision) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (!(tol > 0 && tol < 1)) return fail(NCE_EINVAL, "tol_gmres must lie in (0, 1)");
    if (max_iter < 1 || max_iter > 2000) return fail(NCE_EINVAL, "max_iter must lie in [1, 2000]");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        if (max_iter + 8 > (int)ctx->d_h.n) {
            ctx->d_h.alloc((size_t)max_iter + 8);
            ctx->d_partial.alloc((size_t)nce::kReduceBlocks * ((size_t)max_iter + 8));
        }
        ctx->opts.tol_gmres = tol;
        ctx->opts.max_iter = max_iter;
        ctx->opts.precision = precision;
        return NCE_OK;
    });
}

int nce_solve_interior(nce_ctx* ctx, double* coeffs, double* flux, double* mfpt, nce_info* info) {
    if (!ctx || !mfpt) return fail(NCE_EINVAL, "NULL argument");
    if (ctx->tab.problem != NCE_INTERIOR) return fail(NCE_ESTATE, "context was built for the exterior problem");
    return guarded([&]() -> int {
        double Is = 0;
        int rc = solve(ctx, coeffs, flux, &Is, info);
        *mfpt = 1.0 / (3.0 * Is) - 0.6;
        return rc;
    });
}

int nce_solve_exterior(nce_ctx* ctx, double* coeffs, double* flux, double* rate, double* Is_out, nce_info* info) {
    if (!ctx || !rate) return fail(NCE_EINVAL, "NULL argument");
    if (ctx->tab.problem != NCE_EXTERIOR) return fail(NCE_ESTATE, "context was built for the interior problem");
    return guarded([&]() -> int {
        double Is = 0;
        int rc = solve(ctx, coeffs, flux, &Is, info);
        *rate = 4.0 * M_PI * Is;
        if (Is_out) *Is_out = Is;
        return rc;
    });
}

int nce_mlp_create(int n_in, int width, int hidden, int n_out, uint64_t seed, nce_mlp** out) {
    if (!out) return fail(NCE_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_in < 1 || n_out < 1 || hidden < 0 || (hidden > 0 && width < 1) || hidden > 16)
        return fail(NCE_EINVAL, "bad network shape");
    return guarded([&]() -> int {
        *out = new nce_mlp(n_in, width, hidden, n_out, seed);
        return NCE_OK;
    });
}

void nce_mlp_destroy(nce_mlp* m) { delete m; }

int nce_mlp_num_params(const nce_mlp* m, int64_t* n) {
    if (!m || !n) return fail(NCE_EINVAL, "NULL argument");
    *n = m->net.nparam;
    return NCE_OK;
}

int nce_mlp_get_params(const nce_mlp* m, float* h) {
    if (!m || !h) return fail(NCE_EINVAL, "NULL argument");
    return guarded([&]() -> int {
        HIPCHK(hipMemcpy(h, m->net.theta, sizeof(float) * m->net.nparam, hipMemcpyDeviceToHost));
        return NCE_OK;
    });
}

int nce_mlp_set_params(nce_mlp* m, const float* h) {
    if (!m || !h) return fail(NCE_EINVAL, "NULL argument");
    for (int64_t q = 0; q < m->net.nparam; ++q)
        if (!std::isfinite(h[q])) return fail(NCE_EINVAL, "non-finite network parameter");
    return guarded([&]() -> int {
        HIPCHK(hipMemcpy(m->net.theta, h, sizeof(float) * m->net.nparam, hipMemcpyHostToDevice));
        m->net.step = 0;
        HIPCHK(hipMemset(m->net.mom, 0, sizeof(float) * m->net.nparam));
        HIPCHK(hipMemset(m->net.vel, 0, sizeof(float) * m->net.nparam));
        return NCE_OK;
    });
}

int nce_mlp_forward(nce_mlp* m, const float* x, int64_t B, float* y, void* stream) {
    if (!m || !x || !y || B < 1) return fail(NCE_EINVAL, "bad argument");
    return guarded([&]() -> int {
        hipStream_t s = (hipStream_t)stream;
        const float* out = m->net.forward(s, x, B);
        HIPCHK(hipMemcpyAsync(y, out, sizeof(float) * B * m->net.n_out, hipMemcpyDeviceToDevice, s));
        return NCE_OK;
    });
}

// ---- network forward pass without allocation ------------------------------
// Workspace of nce_mlp_forward_noalloc: a fixed device array (16 MiB on every
// GPU the library runs on, held until the process ends). Host code never
// passes its name to a kernel: the name is a host-side stand-in; the device
// address of each GPU's copy comes from hipGetSymbolAddress.
static constexpr int64_t kNoallocFloats = (int64_t)4 << 20;
static __device__ __align__(256) float scratch[kNoallocFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current GPU's copy of `scratch`, looked up once per
// device with that device current.
float* scratch_on_current_device() {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw HipError("device index beyond the workspace table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<float*>(ptr);
    }
    return g_scratch_ptr[dev];
}
}  // namespace

int nce_mlp_forward_noalloc(nce_mlp* m, const float* x, int64_t B, float* y, void* stream) {
    if (!m || !x || !y || B < 1) return fail(NCE_EINVAL, "bad argument");
    if (2 * m->net.widest_hidden() > kNoallocFloats)
        return fail(NCE_EINVAL, "hidden layers wider than the fixed workspace holds (2 x width floats per row, 16 MiB)");
    return guarded([&]() -> int {
        float* ws = scratch_on_current_device();
        m->net.forward_ws((hipStream_t)stream, x, B, y, ws, kNoallocFloats);
        return NCE_OK;
    });
}

int nce_mlp_loss_grad(nce_mlp* m, const float* x, const float* t, int64_t B, double* loss, float* grad, void* stream) {
    if (!m || !x || !t || B < 1) return fail(NCE_EINVAL, "bad argument");
    return guarded([&]() -> int {
        hipStream_t s = (hipStream_t)stream;
        m->net.loss_grad(s, x, t, B);
        if (loss) {
            double v = 0;
            HIPCHK(hipMemcpyAsync(&v, m->net.lossd, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            *loss = v / ((double)B * m->net.n_out);
        }
        if (grad) {
            HIPCHK(hipMemcpyAsync(grad, m->net.grad, sizeof(float) * m->net.nparam, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        return NCE_OK;
    });
}

int nce_mlp_train_step(nce_mlp* m, const float* x, const float* t, int64_t B, float lr, double* loss, void* stream) {
    if (!m || !x || !t || B < 1 || !(lr > 0)) return fail(NCE_EINVAL, "bad argument");
    return guarded([&]() -> int {
        hipStream_t s = (hipStream_t)stream;
        m->net.loss_grad(s, x, t, B);
        m->net.adam_step(s, lr);
        if (loss) {
            double v = 0;
            HIPCHK(hipMemcpyAsync(&v, m->net.lossd, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            *loss = v / ((double)B * m->net.n_out);
        }
        return NCE_OK;
    });
}

int nce_features(nce_ctx* ctx, float* feat) {
    if (ctx && ctx->ntype > 1) return fail(NCE_ESTATE, "not available for a layout of several patch radii");
    if (!ctx || !feat) return fail(NCE_EINVAL, "NULL argument");
    return guarded([&]() -> int {
        const std::vector<float> f = features_host(ctx);
        HIPCHK(hipMemcpyAsync(feat, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return NCE_OK;
    });
}

int nce_set_deflation(nce_ctx* ctx, int on) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (on != 0 && on != 1) return fail(NCE_EINVAL, "on must be 0 or 1");
    ctx->opts.deflation = on;
    return NCE_OK;
}

int nce_deflation_matrix(nce_ctx* ctx, int* k, double* T_host) {
    if (!ctx || !k) return fail(NCE_EINVAL, "ctx and k must not be NULL");
    return guarded([&]() -> int {
        ensure_deflation(ctx);
        *k = ctx->defl ? ctx->defl->k : 0;
        if (T_host && ctx->defl) std::copy(ctx->defl->T.begin(), ctx->defl->T.end(), T_host);
        return NCE_OK;
    });
}

int nce_coarse_solve(nce_ctx* ctx, double* a, int* iters, double* chi0) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    return guarded([&]() -> int {
        const double* d = coarse_amplitudes(ctx);
        if (a && ctx->ntype > 1)
            HIPCHK(nce::permute_rows(ctx->stream, ctx->N, 1, ctx->d_perm.p, d, a, 1));
        else if (a)
            HIPCHK(hipMemcpyAsync(a, d, sizeof(double) * ctx->N, hipMemcpyDeviceToDevice, ctx->stream));
        if (iters) *iters = ctx->coarse_iters;
        if (chi0 && ctx->ntype > 1)
            for (int t = 0; t < ctx->ntype; ++t) chi0[t] = table_chi0(ctx->tabs[t]);
        else if (chi0)
            *chi0 = ctx->coarse->chi0;
        HIPCHK(hipStreamSynchronize(ctx->stream));
        return NCE_OK;
    });
}

int nce_set_warm_start(nce_ctx* ctx, nce_mlp* m, int use_coarse) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    if (m && ctx->ntype > 1)
        return fail(NCE_ESTATE, "the network's features are for one patch radius: use the coarse start alone");
    if (m && (m->net.n_in != nce::kFeatureDim || m->net.n_out != ctx->K))
        return fail(NCE_ESTATE, "network shape does not match NCE_FEATURES -> K");
    if (m && !use_coarse) return fail(NCE_EINVAL, "the network refines the coarse solve: use_coarse must be 1");
    return guarded([&]() -> int {
        ctx->warm = m ? &m->net : nullptr;
        ctx->warm_coarse = use_coarse != 0;
        if (!m && !use_coarse) {
            // disabled: drop the per-layout data, so a later start recomputes it
            ctx->d_feat.release();
            ctx->d_a.release();
            ctx->coarse_iters = -1;
            return NCE_OK;
        }
        // per-layout preprocessing now, not inside the next solve
        if (ctx->warm && ctx->N > 1 && !ctx->d_feat.p) {
            // the neighbour features on host threads while the coarse solve runs
            // on the device; the amplitude features follow from its result
            std::vector<float> feat;
            auto geometry = std::async(std::launch::async, [&] {
                nce::patch_features_geometry(ctx->frames, ctx->N, ctx->eps, ctx->tab.problem, feat);
            });
            coarse_amplitudes(ctx);
            geometry.get();
            std::vector<double> ah((size_t)ctx->N);
            HIPCHK(hipMemcpyAsync(ah.data(), ctx->d_a.p, sizeof(double) * ah.size(), hipMemcpyDeviceToHost,
                                  ctx->stream));
            HIPCHK(hipStreamSynchronize(ctx->stream));
            nce::patch_features_amplitudes(ah, ctx->N, feat);
            ctx->d_feat.upload(feat, ctx->stream);
        } else if (ctx->warm_coarse && ctx->N > 1) {
            coarse_amplitudes(ctx);
        }
        return NCE_OK;
    });
}

int nce_integral_vector(const nce_ctx* ctx, double* I) {
    if (!ctx || !I) return fail(NCE_EINVAL, "NULL argument");
    if (ctx->ntype > 1) return fail(NCE_ESTATE, "several patch radii: use nce_types for each radius's vector");
    std::memcpy(I, ctx->tab.I.data(), sizeof(double) * ctx->K);
    return NCE_OK;
}

const char* nce_strerror(int code) {
    switch (code) {
        case NCE_OK: return "ok";
        case NCE_NOTCONVERGED: return "iteration limit reached before the tolerance";
        case NCE_EINVAL: return "invalid argument";
        case NCE_ESEP: return "patches closer than 3 eps";
        case NCE_ENOMEM: return "out of memory";
        case NCE_EHIP: return "HIP runtime error";
        case NCE_ETABLE: return "precompute failed its self-check";
        case NCE_ESTATE: return "call not valid in this state";
        default: return "unknown status";
    }
}

const char* nce_last_error(void) { return g_err.c_str(); }

}  // extern "C"
