// Private to the library: the solver context and the pieces of its
// implementation shared by the single-configuration and batched entry points.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/nce.h"
#include "coarse.hpp"
#include "deflate.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "precompute.hpp"
#include "precompute_gpu.hpp"
#include "tree.hpp"

namespace nce_detail {

extern thread_local std::string g_err;

inline int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_));                    \
    } while (0)

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept : p(o.p), n(o.n) {
        o.p = nullptr;
        o.n = 0;
    }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        if (hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) {
            p = nullptr;
            throw std::bad_alloc();
        }
        n = count;
    }
    void upload(const std::vector<T>& v, hipStream_t s) {
        alloc(v.size());
        if (n) {
            HIPCHK(hipMemcpyAsync(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));  // the host vector may be a temporary
        }
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    ~DevBuf() { release(); }
};

template <class T>
inline std::vector<float> to_f32(const std::vector<T>& v) {
    return std::vector<float>(v.begin(), v.end());
}


}  // namespace nce_detail

using nce_detail::DevBuf;

struct nce_ctx {
    nce_opts opts;
    int64_t N = 0;
    int K = 0, Kstar = 0, p = 0;
    int ptot = 0;                       // strengths per patch over all outgoing tables in use
    std::vector<int> tab_off, tab_p;    // per table: first column and size (table 0 = base)
    // outgoing tables of the FP32 applies (opts.tol_id_fp32; the same as above when equal to tol_id)
    bool has_tab32 = false;
    nce::PatchTables tab32;
    int p32 = 0, ptot32 = 0;
    std::vector<int> tab_off32, tab_p32;
    double eps = 0;
    nce::PatchTables tab;
    std::vector<double> frames;  // N x 9: c, e1, e2
    // independent configurations sharing (problem, eps): patches of
    // configuration c are [cfg_first[c], cfg_first[c + 1]); they never interact
    std::vector<int64_t> cfg_first;
    std::vector<char> cfg_tree;         // per configuration: far field by the tree (1) or directly (0)
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool use_tree = false;              // tree pipeline (also used by a multi-configuration context)
    // kernel shapes chosen by autotune() per precision (0 FP64, 1 FP32):
    // P2L grid points per thread and interpolation nodes per thread
    int tune_p2l[2] = {4, 4};
    int tune_l2t[2] = {2, 2};
    nce::Tree tree;
    nce::DeviceTree dtree;
    // grids of the FP32 applies at opts.tol_grid_fp32 (when it differs from tol_grid)
    bool has_tree32 = false;
    nce::Tree tree32;
    nce::DeviceTree dtree32;
    // device tables
    DevBuf<double> d_frames, d_T, d_P, d_I, d_node_off, d_skel_off;
    DevBuf<float> d_T32, d_P32, d_node_off32, d_skel_off32;
    // P's factors (transform_factors) for the interpolation kernel's fused P apply
    DevBuf<double> d_Ptrig, d_Prad;
    DevBuf<float> d_Ptrig32, d_Prad32;
    DevBuf<int> d_Pmode;
    int trig_ld = 0;                    // row stride of d_Ptrig(32)
    DevBuf<nce::LogEntry> d_logtab;     // FP64 logarithm table of the direct sums
    // matvec work arrays
    DevBuf<double> d_rho, d_U;
    DevBuf<float> d_rho32, d_U32, d_x32;
    // solver work arrays
    DevBuf<double> d_V, d_b, d_r, d_x, d_h, d_partial, d_scal;
    int vcap = 0;  // number of Krylov vectors allocated
    // initial guess: monopole (coarse) solve, optionally refined per patch by
    // the learned network (x0_i = a_i m_i)
    bool warm_coarse = false;
    nce::Mlp* warm = nullptr;
    std::unique_ptr<nce::CoarseSolver> coarse;
    DevBuf<double> d_a;                 // coarse amplitudes a_i (valid when coarse_iters >= 0)
    // the coarse model's apply through the tree: one-point tables and one node
    // per patch (zero offsets, unit sizes), the FP32 charges and summed field
    DevBuf<int> d_ctab_off, d_ctab_p;
    DevBuf<float> d_c0, d_cq, d_cu;
    int coarse_iters = -1;
    DevBuf<float> d_feat;
    // coarse-space deflation of the FP32 inner solves (built at the first mixed solve)
    std::unique_ptr<nce::Deflation> defl;
    DevBuf<double> d_dtmp;
    // several patch radii (ntype > 1): patches are held sorted by radius; the
    // context's patch a is the caller's patch perm[a], and patches of type t
    // are [type_first[t], type_first[t + 1])
    int ntype = 1;
    std::vector<double> type_eps;
    std::vector<int64_t> type_first;
    std::vector<int64_t> perm;
    std::vector<nce::PatchTables> tabs, tabs32;
    nce::TypeLayout tl, tl32;                 // per-(type, table) skeleton starts, columns, sizes
    std::vector<int> type_Toff, type_Toff32;  // first row of each type's tables in d_T / d_T32
    std::vector<int> type_ptot, type_ptot32;  // strengths per patch of each type
    int ldr = 0, ldr32 = 0;                   // row length of rho / rho32
    DevBuf<int64_t> d_perm;
    DevBuf<int> d_ptype, d_tsoff, d_tcol, d_tp, d_tsoff32, d_tcol32, d_tp32;
    DevBuf<double> d_Ityp;                    // ntype x K integral vectors
    DevBuf<double> d_xp, d_yp, d_fluxp;       // vectors in the context's order
};

struct nce_mlp {
    nce::Mlp net;
    nce_mlp(int a, int b, int c, int d, uint64_t e) : net(a, b, c, d, e) {}
};

namespace nce_detail {

template <class F>
int guarded(F&& f) {
    try {
        return f();
    } catch (const HipError& e) {
        return fail(NCE_EHIP, e.what());
    } catch (const std::bad_alloc&) {
        return fail(NCE_ENOMEM, "allocation failed");
    } catch (const std::exception& e) {
        return fail(NCE_ETABLE, e.what());
    }
}


// Fills a context for the configurations [cfg_first[c], cfg_first[c + 1]) of
// centers (all with the same eps and opts.problem). forest = false: one
// configuration, far field chosen by opts.far_field (automatic: tree above
// 4000 patches). forest = true: several configurations, each summed by its own
// tree or directly (opts.far_field, or the cheaper by operation count).
void init_ctx(nce_ctx* ctx, const double* centers, const std::vector<int64_t>& cfg_first, double eps,
              const nce_opts& o, bool forest);
// Checks option ranges.
int validate_opts(const nce_opts& o, double eps);
// Patch frames (c, e1, e2 per patch) of unit centres.
void build_frames(const double* c, int64_t N, std::vector<double>& fr);
// uploads P's factors for the fused P apply (enqueued on s)
void upload_transform_factors(nce_ctx* ctx, hipStream_t s);
// Fills a context for one configuration of several patch radii (radius[i] of
// patch i, at least two distinct values).
void init_ctx_types(nce_ctx* ctx, const double* centers, const double* radius, int64_t N, const nce_opts& o);
// Checks unit centres and 3 eps separation within every configuration.
int validate_centers(const double* centers, const std::vector<int64_t>& cfg_first, double eps);
// y = A x (FP64 in and out; precision selects the FP64 or FP32 apply),
// enqueued on ctx->stream; no host synchronisation. live (device, may be
// null): per configuration of a multi-configuration context, 0 skips that
// configuration's Green's-function work (its rows of y are then unspecified).
void matvec(nce_ctx* ctx, const double* x, double* y, int precision, hipEvent_t* ev = nullptr,
            const int* live = nullptr);
// Coarse amplitudes a (device, N) of the context's layout, solved once and kept.
const double* coarse_amplitudes(nce_ctx* ctx);
// Host copy of the network features (kFeatureDim per patch).
std::vector<float> features_host(nce_ctx* ctx);
// Times every valid shape of the P2L and interpolation kernels on the
// context's own tree at the given precision and keeps the fastest
// (synchronises the stream; no-op without a tree).
void autotune(nce_ctx* ctx, int precision);

}  // namespace nce_detail
