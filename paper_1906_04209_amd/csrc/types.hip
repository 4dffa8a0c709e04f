// Several patch radii in one configuration. The paper's formulation (Sections
// 3, 6 and 8) carries over with one set of per-eps tables per radius: patch j
// radiates through its own radius's outgoing representation, patch i is
// sampled at its own radius's Zernike nodes, and P (which acts on functions of
// t/eps) is shared. Patches are held sorted by radius inside the context, so
// that the block apply is one GEMM per radius over a contiguous range of
// patches; the entry points permute coefficient vectors at the boundary.
//
// The tree is built with the largest radius (its caps and validity distances
// bound every smaller patch's), and every radius's recompressions sit at the
// largest radius's ladder distances D_k = 2 eps_max 2^(k/2), so a grid's
// outgoing-table index is valid for sources of every radius; P2L work items
// carry sources of one radius each.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <unordered_map>
#include <vector>

#include "ctx.hpp"

using namespace nce_detail;

namespace nce_detail {

// Patches i, j closer than eps_i + eps_j + max(eps_i, eps_j) in arclength ->
// NCE_ESEP (grid hash with cells of the largest such distance).
static int check_separation_types(const double* c, const double* radius, int64_t N) {
    double rmax = 0.0;
    for (int64_t i = 0; i < N; ++i) rmax = std::max(rmax, radius[i]);
    const double sepmax = 3.0 * rmax;
    const double h = std::max(2.0 * std::sin(std::min(sepmax, M_PI) / 2.0) * (1.0 + 1e-9), 1e-12);
    const int64_t ncell = (int64_t)std::ceil(2.0 / h) + 2;
    auto key = [&](int64_t x, int64_t y, int64_t z) { return (x * ncell + y) * ncell + z; };
    std::unordered_map<int64_t, std::vector<int64_t>> cells;
    std::vector<int64_t> cx(N), cy(N), cz(N);
    for (int64_t i = 0; i < N; ++i) {
        cx[i] = (int64_t)std::floor((c[3 * i] + 1.0) / h);
        cy[i] = (int64_t)std::floor((c[3 * i + 1] + 1.0) / h);
        cz[i] = (int64_t)std::floor((c[3 * i + 2] + 1.0) / h);
        cells[key(cx[i], cy[i], cz[i])].push_back(i);
    }
    for (int64_t i = 0; i < N; ++i)
        for (int64_t a = -1; a <= 1; ++a)
            for (int64_t b = -1; b <= 1; ++b)
                for (int64_t d = -1; d <= 1; ++d) {
                    auto it = cells.find(key(cx[i] + a, cy[i] + b, cz[i] + d));
                    if (it == cells.end()) continue;
                    for (int64_t j : it->second) {
                        if (j <= i) continue;
                        const double* p = c + 3 * i;
                        const double* q = c + 3 * j;
                        const double x = p[1] * q[2] - p[2] * q[1], y = p[2] * q[0] - p[0] * q[2],
                                     z = p[0] * q[1] - p[1] * q[0];
                        const double ang = std::atan2(std::sqrt(x * x + y * y + z * z),
                                                      p[0] * q[0] + p[1] * q[1] + p[2] * q[2]);
                        const double need = radius[i] + radius[j] + std::max(radius[i], radius[j]);
                        if (ang < need * (1.0 - 1e-12))
                            return fail(NCE_ESEP, "patches " + std::to_string(i) + " and " + std::to_string(j) +
                                                      " are closer than eps_i + eps_j + max(eps_i, eps_j)");
                    }
                }
    return NCE_OK;
}

// Concatenated outgoing tables of every radius (the base table, then the
// ladder when the tree is used): T rows, skeleton offsets, and per (type,
// table) the skeleton start, the column in a patch's strength row and the size.
static void layout_types(const std::vector<nce::PatchTables>& tabs, bool ladder, std::vector<double>& Tall,
                         std::vector<double>& soff, nce::TypeLayout& tl, std::vector<int>& Toff,
                         std::vector<int>& ptot, int& ldr, int& pmax) {
    const int ntype = (int)tabs.size();
    tl.ntab = ladder ? 1 + (int)tabs[0].far.size() : 1;
    tl.t_soff.clear();
    tl.t_col.clear();
    tl.t_p.clear();
    Tall.clear();
    soff.clear();
    Toff.assign(ntype, 0);
    ptot.assign(ntype, 0);
    ldr = pmax = 0;
    for (int ty = 0; ty < ntype; ++ty) {
        const nce::PatchTables& t = tabs[ty];
        if ((int)t.far.size() + 1 < tl.ntab) throw std::runtime_error("radius tables with different ladders");
        Toff[ty] = (int)(Tall.size() / t.K);
        int col = 0;
        for (int k = 0; k < tl.ntab; ++k) {
            const std::vector<double>& T = k == 0 ? t.T : t.far[k - 1].T;
            const std::vector<double>& so = k == 0 ? t.skel_off : t.far[k - 1].skel_off;
            const int p = k == 0 ? t.p : t.far[k - 1].p;
            tl.t_soff.push_back((int)(soff.size() / 3));
            tl.t_col.push_back(col);
            tl.t_p.push_back(p);
            Tall.insert(Tall.end(), T.begin(), T.end());
            soff.insert(soff.end(), so.begin(), so.end());
            col += p;
        }
        ptot[ty] = col;
        ldr = std::max(ldr, col);
        pmax = std::max(pmax, t.p);
    }
}

void init_ctx_types(nce_ctx* ctx, const double* centers, const double* radius, int64_t N, const nce_opts& o) {
    ctx->opts = o;
    ctx->N = N;
    ctx->cfg_first = {0, N};
    // distinct radii in ascending order = types; patches sorted by type (stable)
    std::vector<double> radii(radius, radius + N);
    std::sort(radii.begin(), radii.end());
    radii.erase(std::unique(radii.begin(), radii.end()), radii.end());
    ctx->ntype = (int)radii.size();
    ctx->type_eps = radii;
    std::vector<int> ty(N);
    for (int64_t i = 0; i < N; ++i)
        ty[i] = (int)(std::lower_bound(radii.begin(), radii.end(), radius[i]) - radii.begin());
    ctx->perm.resize(N);
    for (int64_t i = 0; i < N; ++i) ctx->perm[i] = i;
    std::stable_sort(ctx->perm.begin(), ctx->perm.end(), [&](int64_t a, int64_t b) { return ty[a] < ty[b]; });
    std::vector<double> cint((size_t)3 * N);
    ctx->tl.ptype.resize(N);
    ctx->type_first.assign(ctx->ntype + 1, 0);
    for (int64_t a = 0; a < N; ++a) {
        const int64_t i = ctx->perm[a];
        for (int d = 0; d < 3; ++d) cint[3 * a + d] = centers[3 * i + d];
        ctx->tl.ptype[a] = ty[i];
        ctx->type_first[ty[i] + 1] = a + 1;
    }
    const double emax = radii.back();
    ctx->eps = emax;
    if (o.stream) {
        ctx->stream = (hipStream_t)o.stream;
    } else {
        HIPCHK(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking));
        ctx->own_stream = true;
    }
    hipStream_t s = ctx->stream;
    std::string dir;
    if (o.cache_dir) dir = o.cache_dir;
    else if (const char* e = std::getenv("NCE_CACHE")) dir = e;
    std::unique_ptr<nce::PrecomputeDevice> pdev;
    {
        const char* hp = std::getenv("NCE_HOST_PRECOMPUTE");
        if (!(hp && hp[0] == '1')) pdev = nce::make_gpu_precompute(s);
    }
    const double tid32 = o.tol_id_fp32 > 0 ? o.tol_id_fp32 : o.tol_id;
    ctx->has_tab32 = tid32 != o.tol_id;
    auto get = [&](double eps, double tid) {
        nce::PatchTables t;
        if (!nce::load_tables(dir, o.problem, eps, o.M, tid, t, emax)) {
            t = nce::build_tables(o.problem, eps, o.M, tid, 0, pdev.get(), emax);
            nce::save_tables(dir, t);
        }
        return t;
    };
    for (double e : radii) {
        ctx->tabs.push_back(get(e, o.tol_id));
        ctx->tabs32.push_back(ctx->has_tab32 ? get(e, tid32) : ctx->tabs.back());
    }
    // shared quantities from the largest radius (K, K*, P, the problem; the
    // tree is built with its caps and ladder)
    ctx->tab = ctx->tabs.back();
    ctx->tab32 = ctx->tabs32.back();
    ctx->K = ctx->tab.K;
    ctx->Kstar = ctx->tab.Kstar;
    build_frames(cint.data(), N, ctx->frames);
    // far field: the tree or all pairs, as for one radius (by the largest)
    if (N < 2 || o.far_field == NCE_FAR_DIRECT) {
        ctx->use_tree = false;
    } else {
        nce::build_tree(ctx->frames, N, emax, ctx->tab, o.tol_grid, ctx->tree);
        const double direct = (double)N * (double)(N - 1) * ctx->Kstar * (double)ctx->tab.p;
        const double viatree = ctx->tree.pairs_far + ctx->tree.pairs_near + 0.25 * ctx->tree.interp_fma;
        ctx->use_tree = o.far_field == NCE_FAR_TREE || viatree < direct;
        if (!ctx->use_tree) ctx->tree = nce::Tree();
    }
    std::vector<double> Tall, soff, Tall32, soff32;
    layout_types(ctx->tabs, ctx->use_tree, Tall, soff, ctx->tl, ctx->type_Toff, ctx->type_ptot, ctx->ldr, ctx->p);
    ctx->tl32.ptype = ctx->tl.ptype;
    layout_types(ctx->tabs32, ctx->use_tree, Tall32, soff32, ctx->tl32, ctx->type_Toff32, ctx->type_ptot32,
                 ctx->ldr32, ctx->p32);
    ctx->tl.node_stride = ctx->tl32.node_stride = 3 * ctx->Kstar;
    ctx->ptot = ctx->ldr;
    ctx->ptot32 = ctx->ldr32;
    std::vector<double> noff, Ity;
    for (const auto& t : ctx->tabs) {
        noff.insert(noff.end(), t.node_off.begin(), t.node_off.end());
        Ity.insert(Ity.end(), t.I.begin(), t.I.end());
    }
    ctx->d_frames.upload(ctx->frames, s);
    ctx->d_T.upload(Tall, s);
    ctx->d_P.upload(ctx->tab.P, s);
    ctx->d_I.upload(ctx->tab.I, s);
    ctx->d_Ityp.upload(Ity, s);
    ctx->d_node_off.upload(noff, s);
    ctx->d_skel_off.upload(soff, s);
    ctx->d_T32.upload(to_f32(Tall32), s);
    ctx->d_P32.upload(to_f32(ctx->tab.P), s);
    upload_transform_factors(ctx, s);
    ctx->d_node_off32.upload(to_f32(noff), s);
    ctx->d_skel_off32.upload(to_f32(soff32), s);
    ctx->d_ptype.upload(ctx->tl.ptype, s);
    ctx->d_tsoff.upload(ctx->tl.t_soff, s);
    ctx->d_tcol.upload(ctx->tl.t_col, s);
    ctx->d_tp.upload(ctx->tl.t_p, s);
    ctx->d_tsoff32.upload(ctx->tl32.t_soff, s);
    ctx->d_tcol32.upload(ctx->tl32.t_col, s);
    ctx->d_tp32.upload(ctx->tl32.t_p, s);
    {
        std::vector<nce::LogEntry> lt(nce::kLogTab);
        nce::build_log_table(lt.data());
        ctx->d_logtab.upload(lt, s);
    }
    std::vector<int64_t> pm(ctx->perm.begin(), ctx->perm.end());
    ctx->d_perm.upload(pm, s);
    const size_t n = (size_t)N * ctx->K;
    ctx->d_rho.alloc((size_t)N * ctx->ldr);
    ctx->d_U.alloc((size_t)N * ctx->Kstar);
    ctx->d_rho32.alloc((size_t)N * ctx->ldr32);
    ctx->d_U32.alloc((size_t)N * ctx->Kstar);
    ctx->d_x32.alloc(n);
    ctx->d_b.alloc(n);
    ctx->d_r.alloc(n);
    ctx->d_x.alloc(n);
    ctx->d_xp.alloc(n);
    ctx->d_yp.alloc(n);
    ctx->d_fluxp.alloc((size_t)N);
    ctx->d_h.alloc((size_t)o.max_iter + 8);
    ctx->d_partial.alloc((size_t)nce::kReduceBlocks * ((size_t)o.max_iter + 8));
    ctx->d_scal.alloc(8);
    ctx->cfg_tree.assign(1, ctx->use_tree ? 1 : 0);
    const double tol32 = o.tol_grid_fp32 > 0 ? o.tol_grid_fp32 : o.tol_grid;
    ctx->has_tree32 = ctx->use_tree && (tol32 != o.tol_grid || ctx->has_tab32);
    if (ctx->use_tree) {
        nce::split_items_by_type(ctx->tree, ctx->tl, ctx->Kstar, ctx->frames, emax, ctx->tab.problem);
        nce::upload_tree(ctx->tree, ctx->Kstar, ctx->p, {}, {}, s, ctx->dtree, &ctx->tl);
    }
    if (ctx->has_tree32) {
        nce::build_tree(ctx->frames, N, emax, ctx->tab32, tol32, ctx->tree32, false);
        nce::split_items_by_type(ctx->tree32, ctx->tl32, ctx->Kstar, ctx->frames, emax, ctx->tab.problem);
        nce::upload_tree(ctx->tree32, ctx->Kstar, ctx->p32, {}, {}, s, ctx->dtree32, &ctx->tl32);
    }
    HIPCHK(hipStreamSynchronize(s));
}

}  // namespace nce_detail

extern "C" {

int nce_setup_radii(const double* centers, const double* radius, int64_t N, const nce_opts* opts_in,
                    nce_ctx** out) {
    g_err.clear();
    if (!out) return fail(NCE_EINVAL, "out is NULL");
    *out = nullptr;
    nce_opts o;
    nce_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (!centers || !radius || N < 1) return fail(NCE_EINVAL, "need N >= 1 centres and radii");
    double rmax = 0.0;
    std::vector<double> distinct;
    for (int64_t i = 0; i < N; ++i) {
        if (!(radius[i] > 0.0 && radius[i] <= M_PI / 3.0))
            return fail(NCE_EINVAL, "radius " + std::to_string(i) + " outside (0, pi/3]");
        rmax = std::max(rmax, radius[i]);
        if (std::find(distinct.begin(), distinct.end(), radius[i]) == distinct.end()) {
            distinct.push_back(radius[i]);
            if (distinct.size() > 8) return fail(NCE_EINVAL, "more than 8 distinct patch radii");
        }
    }
    int rc = validate_opts(o, rmax);
    if (rc != NCE_OK) return rc;
    for (int64_t i = 0; i < N; ++i) {
        const double* c = centers + 3 * i;
        if (!std::isfinite(c[0]) || !std::isfinite(c[1]) || !std::isfinite(c[2]))
            return fail(NCE_EINVAL, "non-finite centre " + std::to_string(i));
        if (std::fabs(std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]) - 1.0) > 1e-12)
            return fail(NCE_EINVAL, "centre " + std::to_string(i) + " is not a unit vector");
    }
    rc = check_separation_types(centers, radius, N);
    if (rc != NCE_OK) return rc;
    return guarded([&]() -> int {
        auto* ctx = new nce_ctx();
        std::unique_ptr<nce_ctx, void (*)(nce_ctx*)> guard(ctx, nce_destroy);
        if (distinct.size() == 1)
            init_ctx(ctx, centers, {0, N}, distinct[0], o, false);
        else
            init_ctx_types(ctx, centers, radius, N, o);
        *out = guard.release();
        return NCE_OK;
    });
}

int nce_types(const nce_ctx* ctx, int* ntypes, double* eps_host, double* I_host, int* type_host) {
    if (!ctx) return fail(NCE_EINVAL, "ctx is NULL");
    const int nt = ctx->ntype;
    if (ntypes) *ntypes = nt;
    for (int t = 0; t < nt; ++t) {
        const double e = nt > 1 ? ctx->type_eps[t] : ctx->eps;
        const std::vector<double>& I = nt > 1 ? ctx->tabs[t].I : ctx->tab.I;
        if (eps_host) eps_host[t] = e;
        if (I_host) std::memcpy(I_host + (size_t)t * ctx->K, I.data(), sizeof(double) * ctx->K);
    }
    if (type_host) {
        if (nt > 1)
            for (int64_t a = 0; a < ctx->N; ++a) type_host[ctx->perm[a]] = ctx->tl.ptype[a];
        else
            std::fill(type_host, type_host + ctx->N, 0);
    }
    return NCE_OK;
}

}  // extern "C"
