// Many independent configurations solved together (C ABI in include/nce.h).
//
// Configurations with the same (problem, eps) share precomputed tables, so
// they are gathered into one group context whose patches are the union of the
// group's configurations and whose far field is a forest: each configuration
// brings its own cube-sphere tree, or all-pairs direct lists where those cost
// fewer operations. One system apply of the batch is then a handful of large
// launches per group (block apply, P2L over every configuration's grids, near
// lists, interpolation, P apply) instead of five small ones per configuration.
//
// Batch vectors are the groups' coefficient vectors one after another;
// configuration b occupies the elements [off[b], off[b] + N_b K).
//
// GMRES runs in lockstep over the configurations: one Krylov index j for all,
// but each configuration has its own Arnoldi coefficients, Givens rotations,
// residual estimate and tolerance, and drops out (its rotations freeze) when
// it converges. Every reduction is segmented by configuration and
// deterministic. One Arnoldi step -- copy of v_j, the batched apply, classical
// Gram-Schmidt twice, the norm, the Givens update and the store of v_{j+1} --
// reads j from device memory, so the whole step is captured once as a HIP
// graph and replayed. The host only reads the convergence flags between steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <numeric>
#include <vector>

#include "ctx.hpp"

using namespace nce_detail;

namespace {

constexpr int kChunk = 16384;   // vector elements per reduction chunk (never straddles configurations)
constexpr int kMaxBatchIter = 120;

__device__ __forceinline__ double block_reduce(double v, double* red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x % 64, wid = threadIdx.x / 64;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

// partial[c * ldp + v] = sum over chunk c of V_v . w, v < nv = (jdev ? *jdev : 0) + add;
// chunks of inactive configurations are skipped.
__global__ __launch_bounds__(256) void k_seg_dots(const double* __restrict__ V, int64_t ldv,
                                                  const double* __restrict__ w, const int* __restrict__ jdev, int add,
                                                  const int64_t* __restrict__ ch_e0, const int* __restrict__ ch_seg,
                                                  const int* __restrict__ active, double* __restrict__ partial,
                                                  int ldp) {
    __shared__ double red[4];
    const int c = blockIdx.x;
    if (!active[ch_seg[c]]) return;
    const int nv = (jdev ? *jdev : 0) + add;
    const int64_t e0 = ch_e0[c], e1 = ch_e0[c + 1];
    for (int v = 0; v < nv; ++v) {
        const double* Vv = V + (int64_t)v * ldv;
        double s = 0.0;
        for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) s += Vv[e] * w[e];
        s = block_reduce(s, red);
        if (threadIdx.x == 0) partial[(int64_t)c * ldp + v] = s;
    }
}

// out[s * ldo + v] = sum of the partials of configuration s's chunks, in order.
__global__ __launch_bounds__(128) void k_seg_reduce(const double* __restrict__ partial, int ldp,
                                                    const int* __restrict__ seg_ch, const int* __restrict__ jdev,
                                                    int add, const int* __restrict__ active, double* __restrict__ out,
                                                    int ldo) {
    const int s = blockIdx.x, v = threadIdx.x;
    const int nv = (jdev ? *jdev : 0) + add;
    if (!active[s] || v >= nv) return;
    double t = 0.0;
    for (int c = seg_ch[s]; c < seg_ch[s + 1]; ++c) t += partial[(int64_t)c * ldp + v];
    out[(int64_t)s * ldo + v] = t;
}

// w -= sum_{v < nv} h[s][v] V_v on the chunks of active configurations
__global__ __launch_bounds__(256) void k_seg_axpys(const double* __restrict__ V, int64_t ldv,
                                                   const int* __restrict__ jdev, int add, const double* __restrict__ h,
                                                   int ldh, const int64_t* __restrict__ ch_e0,
                                                   const int* __restrict__ ch_seg, const int* __restrict__ active,
                                                   double* __restrict__ w) {
    __shared__ double hs[kMaxBatchIter + 8];
    const int c = blockIdx.x, s = ch_seg[c];
    if (!active[s]) return;
    const int nv = (jdev ? *jdev : 0) + add;
    for (int v = threadIdx.x; v < nv; v += blockDim.x) hs[v] = h[(int64_t)s * ldh + v];
    __syncthreads();
    const int64_t e0 = ch_e0[c], e1 = ch_e0[c + 1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        double acc = w[e];
        for (int v = 0; v < nv; ++v) acc -= hs[v] * V[(int64_t)v * ldv + e];
        w[e] = acc;
    }
}

// y = x * scal[s] on active configurations; y = V_{*jdev + 1} when V != nullptr
__global__ __launch_bounds__(256) void k_seg_scale(const double* __restrict__ x, const double* __restrict__ scal,
                                                   const int64_t* __restrict__ ch_e0, const int* __restrict__ ch_seg,
                                                   const int* __restrict__ active, double* __restrict__ y,
                                                   const int* __restrict__ jdev, int64_t ldv) {
    const int c = blockIdx.x, s = ch_seg[c];
    if (!active[s]) return;
    const double a = scal[s];
    double* out = jdev ? y + (int64_t)(*jdev + 1) * ldv : y;
    const int64_t e0 = ch_e0[c], e1 = ch_e0[c + 1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) out[e] = a * x[e];
}

// xin = V_{*jdev}
__global__ void k_copy_vj(const double* __restrict__ V, int64_t ldv, const int* __restrict__ jdev, int64_t n,
                          double* __restrict__ xin) {
    const double* src = V + (int64_t)(*jdev) * ldv;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        xin[e] = src[e];
}

// One Givens step per active configuration s at Krylov index j = *jdev.
// Column of the Hessenberg matrix: h1 + h2 (the two Gram-Schmidt passes; h2
// null after a single pass),
// subdiagonal sqrt(nrm2). Rotations cs/sn (nseg x maxit), triangular factor R
// (nseg x maxit x maxit), right-hand side g (nseg x (maxit + 1)).
__global__ void k_givens(int nseg, const int* __restrict__ jdev, const double* __restrict__ h1,
                         const double* __restrict__ h2, int ldh, const double* __restrict__ nrm2,
                         const double* __restrict__ beta, const double* __restrict__ tol, int maxit,
                         int* __restrict__ active, double* __restrict__ R, double* __restrict__ cs,
                         double* __restrict__ sn, double* __restrict__ g, int* __restrict__ m_used,
                         double* __restrict__ est, double* __restrict__ inv_h) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg || !active[s]) return;
    const int j = *jdev;
    double* Rs = R + (int64_t)s * maxit * maxit;
    double* css = cs + (int64_t)s * maxit;
    double* sns = sn + (int64_t)s * maxit;
    double* gs = g + (int64_t)s * (maxit + 1);
    for (int v = 0; v <= j; ++v)
        Rs[(int64_t)v * maxit + j] = h1[(int64_t)s * ldh + v] + (h2 ? h2[(int64_t)s * ldh + v] : 0.0);
    const double hk1 = sqrt(fmax(nrm2[(int64_t)s * ldh], 0.0));
    for (int v = 0; v < j; ++v) {
        const double a = Rs[(int64_t)v * maxit + j], b = Rs[(int64_t)(v + 1) * maxit + j];
        Rs[(int64_t)v * maxit + j] = css[v] * a + sns[v] * b;
        Rs[(int64_t)(v + 1) * maxit + j] = -sns[v] * a + css[v] * b;
    }
    const double a = Rs[(int64_t)j * maxit + j];
    const double den = hypot(a, hk1);
    const double c = den > 0.0 ? a / den : 1.0, sg = den > 0.0 ? hk1 / den : 0.0;
    css[j] = c;
    sns[j] = sg;
    Rs[(int64_t)j * maxit + j] = den;
    gs[j + 1] = -sg * gs[j];
    gs[j] = c * gs[j];
    const double e = fabs(gs[j + 1]) / beta[s];
    est[s] = e;
    inv_h[s] = hk1 > 0.0 ? 1.0 / hk1 : 0.0;
    const bool happy = hk1 <= 1e-14 * beta[s];
    if (e <= tol[s] || happy || j + 1 >= maxit || den == 0.0) {
        active[s] = 0;
        m_used[s] = den == 0.0 ? j : j + 1;
    }
}

__global__ void k_advance(int* jdev) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *jdev += 1;
}

// y[s][0..m) from R y = g (back substitution), configurations with m_used > 0
__global__ void k_backsolve(int nseg, const double* __restrict__ R, const double* __restrict__ g, int maxit,
                            const int* __restrict__ m_used, double* __restrict__ y) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nseg) return;
    const int m = m_used[s];
    const double* Rs = R + (int64_t)s * maxit * maxit;
    const double* gs = g + (int64_t)s * (maxit + 1);
    double* ys = y + (int64_t)s * maxit;
    for (int i = m - 1; i >= 0; --i) {
        double acc = gs[i];
        for (int k = i + 1; k < m; ++k) acc -= Rs[(int64_t)i * maxit + k] * ys[k];
        ys[i] = acc / Rs[(int64_t)i * maxit + i];
    }
}

// x += sum_{v < m_used[s]} y[s][v] V_v
__global__ __launch_bounds__(256) void k_seg_combine(const double* __restrict__ V, int64_t ldv,
                                                     const double* __restrict__ y, int maxit,
                                                     const int* __restrict__ m_used, const int64_t* __restrict__ ch_e0,
                                                     const int* __restrict__ ch_seg, double* __restrict__ x) {
    __shared__ double ys[kMaxBatchIter + 8];
    const int c = blockIdx.x, s = ch_seg[c];
    const int m = m_used[s];
    if (m == 0) return;
    for (int v = threadIdx.x; v < m; v += blockDim.x) ys[v] = y[(int64_t)s * maxit + v];
    __syncthreads();
    const int64_t e0 = ch_e0[c], e1 = ch_e0[c + 1];
    for (int64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
        double acc = x[e];
        for (int v = 0; v < m; ++v) acc += ys[v] * V[(int64_t)v * ldv + e];
        x[e] = acc;
    }
}

// r = b - r (in place: r holds A x on entry)
__global__ void k_sub_from(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
        r[e] = b[e] - r[e];
}

// b = e_0 on every patch (P 1 in coefficients), x = 0
__global__ void k_init_rhs(int64_t npatch, int K, double* __restrict__ b, double* __restrict__ x) {
    const int64_t n = npatch * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        b[e] = (e % K) == 0 ? 1.0 : 0.0;
        x[e] = 0.0;
    }
}

dim3 grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

}  // namespace

struct nce_batch {
    int B = 0;
    int K = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<nce_ctx*> groups;          // one context per (problem, eps)
    std::vector<int> g_problem;
    std::vector<int64_t> g_elem;           // first vector element of each group (+ total)
    std::vector<int> g_seg0;               // first segment of each group
    std::vector<int> seg_cfg;              // segment (internal order) -> configuration index b
    std::vector<int> cfg_seg;              // configuration b -> segment
    std::vector<int> seg_group;
    std::vector<int64_t> seg_off;          // segment s = elements [seg_off[s], seg_off[s + 1])
    int64_t n = 0;                         // total unknowns
    int nch = 0;
    // reduction chunks
    DevBuf<int64_t> d_ch_e0;
    DevBuf<int> d_ch_seg, d_seg_ch;
    // solver state
    int maxit = 60;
    double tol = 1e-10;
    int precision = NCE_MIXED;
    int use_graph = 1;
    DevBuf<double> d_V, d_xin, d_w, d_b, d_r, d_x, d_flux;
    DevBuf<double> d_partial, d_h1, d_h2, d_nrm, d_beta, d_tol, d_R, d_cs, d_sn, d_g, d_est, d_invh, d_y;
    DevBuf<int> d_active, d_mused, d_j, d_all;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    int graph_maxit[2] = {0, 0};
    bool graph_defl[2] = {false, false};   // whether the captured step applies the deflation
    // initial guess: per-member coarse solves, optionally refined by a network
    bool warm_coarse = false;
    nce::Mlp* warm = nullptr;
    std::vector<DevBuf<double>> g_a;       // per group: coarse amplitudes of its patches
    std::vector<DevBuf<float>> g_feat;     // per group: network features of its patches
    bool have_a = false;
    // coarse-space deflation of the FP32 inner solves, per member (segment order)
    bool deflation = true;
    bool have_defl = false;
    DevBuf<double> d_dZ, d_dM, d_dd, d_dtmp;  // npatch x 16, S x 16 x 16, S x 16, n
    DevBuf<int64_t> d_pseg;                   // S + 1 patch offsets
    DevBuf<int> d_patch_seg;                  // patch -> segment

    ~nce_batch() {
        for (auto& gr : graph)
            if (gr) (void)hipGraphExecDestroy(gr);
        for (nce_ctx* c : groups) nce_destroy(c);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// y = A x for every configuration (batch layout), enqueued on the stream;
// with live (device, per segment) the far-field work of configurations whose
// flag is 0 is skipped.
void batch_matvec(nce_batch* bt, const double* x, double* y, int precision, const int* live = nullptr) {
    for (size_t g = 0; g < bt->groups.size(); ++g)
        matvec(bt->groups[g], x + bt->g_elem[g], y + bt->g_elem[g], precision, nullptr,
               live ? live + bt->g_seg0[g] : nullptr);
}

bool deflated(const nce_batch* bt, int precision) {
    return precision == NCE_MIXED && bt->deflation && bt->have_defl;
}

// Deflation data of every member (built once): bases on host threads over
// all members, one upload, the members' coarse products enqueued back to back
// on shared scratch, one download, then T^{-1} - I per member on the host.
void ensure_batch_deflation(nce_batch* bt) {
    if (bt->have_defl) return;
    hipStream_t s = bt->stream;
    const int S = bt->B;
    const int64_t npatch = bt->n / bt->K;
    std::vector<int64_t> pseg(S + 1);
    std::vector<int> pcfg((size_t)npatch), Nq(S), kq(S);
    std::vector<const double*> frh(S);
    std::vector<double> chi0(S, 0.0);
    int nmax = 1;
    for (int q = 0; q <= S; ++q) pseg[q] = bt->seg_off[q] / bt->K;
    for (int q = 0; q < S; ++q) {
        for (int64_t i = pseg[q]; i < pseg[q + 1]; ++i) pcfg[(size_t)i] = q;
        const int g = bt->seg_group[q];
        nce_ctx* c = bt->groups[g];
        const int member = q - bt->g_seg0[g];
        const int64_t f0 = c->cfg_first[member], nc = c->cfg_first[member + 1] - f0;
        if (nc != pseg[q + 1] - pseg[q]) throw std::runtime_error("batch layout mismatch");
        Nq[q] = (int)nc;
        frh[q] = c->frames.data() + 9 * f0;
        for (int m = 0; m < c->p; ++m) chi0[q] += c->tab.T[(size_t)m * c->K];
        if (nc >= nce::kDeflMinN) nmax = std::max(nmax, (int)nc);
    }
    std::vector<double> Zall((size_t)npatch * nce::kDefl, 0.0), Mall((size_t)S * nce::kDefl * nce::kDefl, 0.0);
    nce::deflation_bases(S, frh.data(), Nq.data(), pseg.data(), nce::kDeflMinN, Zall.data(), kq.data());
    bt->d_dZ.upload(Zall, s);
    DevBuf<double> dS;
    dS.alloc(Zall.size());
    {
        nce::CoarseMultiWs ws;
        ws.reserve(nmax);
        for (int q = 0; q < S; ++q) {
            if (kq[q] == 0) continue;
            const int g = bt->seg_group[q];
            nce_ctx* c = bt->groups[g];
            const int64_t f0 = c->cfg_first[q - bt->g_seg0[g]];
            nce::coarse_multi_enqueue(s, c->tab.problem, Nq[q], c->d_frames.p + 9 * f0,
                                      bt->d_dZ.p + pseg[q] * nce::kDefl, dS.p + pseg[q] * nce::kDefl, ws);
        }
        std::vector<double> Sall(Zall.size());
        HIPCHK(hipMemcpyAsync(Sall.data(), dS.p, sizeof(double) * Sall.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));  // before the scratch is released
        // members with a singular T stay undeflated (their M is zero)
        (void)nce::deflation_inverses(S, Nq.data(), pseg.data(), kq.data(), chi0.data(), Zall.data(), Sall.data(),
                                      Mall.data());
    }
    bt->d_dM.upload(Mall, s);
    bt->d_pseg.upload(pseg, s);
    bt->d_patch_seg.upload(pcfg, s);
    bt->d_dd.alloc((size_t)S * nce::kDefl);
    bt->d_dtmp.alloc((size_t)bt->n);
    HIPCHK(hipStreamSynchronize(s));
    bt->have_defl = true;
}

void drop_graphs(nce_batch* bt) {
    for (auto& gr : bt->graph)
        if (gr) {
            (void)hipGraphExecDestroy(gr);
            gr = nullptr;
        }
}

void ensure_solver(nce_batch* bt, int maxit) {
    if (bt->d_V.n >= (size_t)(maxit + 1) * bt->n && bt->maxit >= maxit && bt->d_R.p) return;
    const int S = bt->B;
    bt->d_V.alloc((size_t)(maxit + 1) * bt->n);
    const int ldp = kMaxBatchIter + 8;
    bt->d_partial.alloc((size_t)bt->nch * ldp);
    bt->d_h1.alloc((size_t)S * ldp);
    bt->d_h2.alloc((size_t)S * ldp);
    bt->d_nrm.alloc((size_t)S * ldp);
    bt->d_beta.alloc(S);
    bt->d_tol.alloc(S);
    bt->d_R.alloc((size_t)S * maxit * maxit);
    bt->d_cs.alloc((size_t)S * maxit);
    bt->d_sn.alloc((size_t)S * maxit);
    bt->d_g.alloc((size_t)S * (maxit + 1));
    bt->d_est.alloc(S);
    bt->d_invh.alloc(S);
    bt->d_y.alloc((size_t)S * maxit);
    bt->d_active.alloc(S);
    bt->d_mused.alloc(S);
    bt->d_all.alloc(S);
    bt->d_j.alloc(1);
    bt->maxit = maxit;
    for (auto& gr : bt->graph)
        if (gr) {
            (void)hipGraphExecDestroy(gr);
            gr = nullptr;
        }
}

// per-configuration squared norms of a batch vector (all configurations) -> host
std::vector<double> seg_norm2(nce_batch* bt, const double* v) {
    hipStream_t s = bt->stream;
    const int ldp = kMaxBatchIter + 8;
    std::vector<int> ones(bt->B, 1);
    HIPCHK(hipMemcpyAsync(bt->d_all.p, ones.data(), sizeof(int) * bt->B, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_seg_dots, dim3(bt->nch), dim3(256), 0, s, v, (int64_t)0, v, (const int*)nullptr, 1,
                       bt->d_ch_e0.p, bt->d_ch_seg.p, bt->d_all.p, bt->d_partial.p, ldp);
    hipLaunchKernelGGL(k_seg_reduce, dim3(bt->B), dim3(128), 0, s, bt->d_partial.p, ldp, bt->d_seg_ch.p,
                       (const int*)nullptr, 1, bt->d_all.p, bt->d_nrm.p, ldp);
    HIPCHK(hipGetLastError());
    std::vector<double> tmp((size_t)bt->B * ldp), out(bt->B);
    HIPCHK(hipMemcpyAsync(tmp.data(), bt->d_nrm.p, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < bt->B; ++q) out[q] = tmp[(size_t)q * ldp];
    return out;
}

// One Arnoldi step at j = *d_j for the active configurations (all launches).
void arnoldi_step(nce_batch* bt, int precision) {
    hipStream_t s = bt->stream;
    const int ldp = kMaxBatchIter + 8;
    const int64_t ldv = bt->n;
    double* V = bt->d_V.p;
    hipLaunchKernelGGL(k_copy_vj, grid_for(bt->n), dim3(256), 0, s, V, ldv, bt->d_j.p, bt->n, bt->d_xin.p);
    // deflated inner solves iterate on A M^{-1}
    if (deflated(bt, precision))
        HIPCHK(nce::deflation_apply_batched(s, bt->B, bt->n / bt->K, bt->K, bt->d_pseg.p, bt->d_patch_seg.p,
                                            bt->d_dZ.p, bt->d_dM.p, bt->d_active.p, bt->d_dd.p, bt->d_xin.p));
    // configurations that have converged (active = 0) skip their sums
    batch_matvec(bt, bt->d_xin.p, bt->d_w.p, precision, bt->d_active.p);
    // classical Gram-Schmidt twice for FP64, once for the FP32 inner solves of
    // the mixed form (their 1e-5 target is far above the orthogonality lost in
    // one pass over FP64 vectors)
    const int passes = precision == NCE_MIXED ? 1 : 2;
    for (int pass = 0; pass < passes; ++pass) {
        double* h = pass == 0 ? bt->d_h1.p : bt->d_h2.p;
        hipLaunchKernelGGL(k_seg_dots, dim3(bt->nch), dim3(256), 0, s, V, ldv, bt->d_w.p, bt->d_j.p, 1,
                           bt->d_ch_e0.p, bt->d_ch_seg.p, bt->d_active.p, bt->d_partial.p, ldp);
        hipLaunchKernelGGL(k_seg_reduce, dim3(bt->B), dim3(128), 0, s, bt->d_partial.p, ldp, bt->d_seg_ch.p,
                           bt->d_j.p, 1, bt->d_active.p, h, ldp);
        hipLaunchKernelGGL(k_seg_axpys, dim3(bt->nch), dim3(256), 0, s, V, ldv, bt->d_j.p, 1, h, ldp,
                           bt->d_ch_e0.p, bt->d_ch_seg.p, bt->d_active.p, bt->d_w.p);
    }
    hipLaunchKernelGGL(k_seg_dots, dim3(bt->nch), dim3(256), 0, s, bt->d_w.p, (int64_t)0, bt->d_w.p,
                       (const int*)nullptr, 1, bt->d_ch_e0.p, bt->d_ch_seg.p, bt->d_active.p, bt->d_partial.p, ldp);
    hipLaunchKernelGGL(k_seg_reduce, dim3(bt->B), dim3(128), 0, s, bt->d_partial.p, ldp, bt->d_seg_ch.p,
                       (const int*)nullptr, 1, bt->d_active.p, bt->d_nrm.p, ldp);
    hipLaunchKernelGGL(k_givens, dim3((bt->B + 63) / 64), dim3(64), 0, s, bt->B, bt->d_j.p, bt->d_h1.p,
                       passes == 2 ? (const double*)bt->d_h2.p : (const double*)nullptr,
                       ldp, bt->d_nrm.p, bt->d_beta.p, bt->d_tol.p, bt->maxit, bt->d_active.p, bt->d_R.p,
                       bt->d_cs.p, bt->d_sn.p, bt->d_g.p, bt->d_mused.p, bt->d_est.p, bt->d_invh.p);
    hipLaunchKernelGGL(k_seg_scale, dim3(bt->nch), dim3(256), 0, s, bt->d_w.p, bt->d_invh.p, bt->d_ch_e0.p,
                       bt->d_ch_seg.p, bt->d_active.p, V, bt->d_j.p, ldv);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, bt->d_j.p);
    HIPCHK(hipGetLastError());
}

// Lockstep GMRES on A d = rhs for the configurations with mask[s] (internal
// segment order), d added into x. Returns per-segment Arnoldi steps and
// residual estimates (relative to ||rhs_s||).
void gmres_batch(nce_batch* bt, const double* rhs, double* x, const std::vector<char>& mask,
                 const std::vector<double>& tol, int precision, std::vector<int>& steps, std::vector<double>& est) {
    hipStream_t s = bt->stream;
    const int S = bt->B, maxit = bt->maxit;
    const std::vector<double> nr2 = seg_norm2(bt, rhs);
    std::vector<int> act(S, 0);
    std::vector<double> beta(S, 1.0), g((size_t)S * (maxit + 1), 0.0), scal(S, 0.0);
    steps.assign(S, 0);
    est.assign(S, 0.0);
    for (int q = 0; q < S; ++q) {
        const double b = std::sqrt(nr2[q]);
        if (mask[q] && b > 0.0) {
            act[q] = 1;
            beta[q] = b;
            g[(size_t)q * (maxit + 1)] = b;
            scal[q] = 1.0 / b;
        }
    }
    if (std::accumulate(act.begin(), act.end(), 0) == 0) return;
    std::vector<int> zero(S, 0);
    HIPCHK(hipMemcpyAsync(bt->d_active.p, act.data(), sizeof(int) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bt->d_mused.p, zero.data(), sizeof(int) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bt->d_beta.p, beta.data(), sizeof(double) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bt->d_tol.p, tol.data(), sizeof(double) * S, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bt->d_g.p, g.data(), sizeof(double) * g.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(bt->d_invh.p, scal.data(), sizeof(double) * S, hipMemcpyHostToDevice, s));
    int j0 = -1;
    HIPCHK(hipMemcpyAsync(bt->d_j.p, &j0, sizeof(int), hipMemcpyHostToDevice, s));
    // v_0 = rhs / beta (written to V_{j0 + 1} = V_0)
    hipLaunchKernelGGL(k_seg_scale, dim3(bt->nch), dim3(256), 0, s, rhs, bt->d_invh.p, bt->d_ch_e0.p,
                       bt->d_ch_seg.p, bt->d_active.p, bt->d_V.p, bt->d_j.p, (int64_t)bt->n);
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, bt->d_j.p);
    HIPCHK(hipGetLastError());
    const int gi = precision == NCE_FP64 ? 0 : 1;
    // the captured step and the final combination must agree on the deflation
    if (bt->graph[gi] && bt->graph_defl[gi] != deflated(bt, precision)) {
        (void)hipGraphExecDestroy(bt->graph[gi]);
        bt->graph[gi] = nullptr;
    }
    if (bt->use_graph && !bt->graph[gi]) {
        hipGraph_t gr = nullptr;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            arnoldi_step(bt, precision);
        } catch (...) {
            (void)hipStreamEndCapture(s, &gr);
            if (gr) (void)hipGraphDestroy(gr);
            throw;
        }
        HIPCHK(hipStreamEndCapture(s, &gr));
        hipGraphExec_t ex = nullptr;
        const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        HIPCHK(e);
        bt->graph[gi] = ex;
        bt->graph_defl[gi] = deflated(bt, precision);
    }
    std::vector<int> a(S);
    for (int j = 0; j < maxit; ++j) {
        if (bt->use_graph) HIPCHK(hipGraphLaunch(bt->graph[gi], s));
        else arnoldi_step(bt, precision);
        HIPCHK(hipMemcpyAsync(a.data(), bt->d_active.p, sizeof(int) * S, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (std::accumulate(a.begin(), a.end(), 0) == 0) break;
    }
    hipLaunchKernelGGL(k_backsolve, dim3((S + 63) / 64), dim3(64), 0, s, S, bt->d_R.p, bt->d_g.p, maxit,
                       bt->d_mused.p, bt->d_y.p);
    if (deflated(bt, precision)) {
        // x += M^{-1} (V y)
        HIPCHK(nce::fill(s, bt->n, 0.0, bt->d_dtmp.p));
        hipLaunchKernelGGL(k_seg_combine, dim3(bt->nch), dim3(256), 0, s, bt->d_V.p, (int64_t)bt->n, bt->d_y.p,
                           maxit, bt->d_mused.p, bt->d_ch_e0.p, bt->d_ch_seg.p, bt->d_dtmp.p);
        HIPCHK(nce::deflation_apply_batched(s, bt->B, bt->n / bt->K, bt->K, bt->d_pseg.p, bt->d_patch_seg.p,
                                            bt->d_dZ.p, bt->d_dM.p, nullptr, bt->d_dd.p, bt->d_dtmp.p));
        HIPCHK(nce::axpby(s, bt->n, 1.0, bt->d_dtmp.p, 1.0, x));
    } else {
        hipLaunchKernelGGL(k_seg_combine, dim3(bt->nch), dim3(256), 0, s, bt->d_V.p, (int64_t)bt->n, bt->d_y.p,
                           maxit, bt->d_mused.p, bt->d_ch_e0.p, bt->d_ch_seg.p, x);
    }
    HIPCHK(hipGetLastError());
    std::vector<double> e(S);
    HIPCHK(hipMemcpyAsync(steps.data(), bt->d_mused.p, sizeof(int) * S, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(e.data(), bt->d_est.p, sizeof(double) * S, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    for (int q = 0; q < S; ++q) est[q] = act[q] ? e[q] : 0.0;
}

// Coarse amplitudes of every member (one coarse solve per member, kept), and
// with a network the features of every patch.
void batch_coarse(nce_batch* bt) {
    if (bt->have_a) return;
    hipStream_t s = bt->stream;
    bt->g_a.resize(bt->groups.size());
    for (size_t g = 0; g < bt->groups.size(); ++g) {
        nce_ctx* c = bt->groups[g];
        double chi0 = 0.0;
        for (int m = 0; m < c->p; ++m) chi0 += c->tab.T[(size_t)m * c->K];
        bt->g_a[g].alloc((size_t)c->N);
        int64_t nmax = 1;
        for (size_t q = 0; q + 1 < c->cfg_first.size(); ++q)
            nmax = std::max<int64_t>(nmax, c->cfg_first[q + 1] - c->cfg_first[q]);
        // one solver for the group, reused by every member
        nce::CoarseSolver cs((int)nmax, c->tab.problem, chi0, 80);
        for (size_t q = 0; q + 1 < c->cfg_first.size(); ++q) {
            const int64_t f0 = c->cfg_first[q], nc = c->cfg_first[q + 1] - f0;
            cs.solve(s, (int)nc, c->d_frames.p + 9 * f0, c->opts.tol_coarse, bt->g_a[g].p + f0);
        }
    }
    bt->have_a = true;
}

void batch_features(nce_batch* bt) {
    if (!bt->g_feat.empty()) return;
    batch_coarse(bt);
    hipStream_t s = bt->stream;
    bt->g_feat.resize(bt->groups.size());
    for (size_t g = 0; g < bt->groups.size(); ++g) {
        nce_ctx* c = bt->groups[g];
        std::vector<double> a((size_t)c->N);
        HIPCHK(hipMemcpyAsync(a.data(), bt->g_a[g].p, sizeof(double) * a.size(), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::vector<float> all;
        all.reserve((size_t)c->N * nce::kFeatureDim);
        for (size_t q = 0; q + 1 < c->cfg_first.size(); ++q) {
            const int64_t f0 = c->cfg_first[q], nc = c->cfg_first[q + 1] - f0;
            std::vector<double> fr(c->frames.begin() + 9 * f0, c->frames.begin() + 9 * (f0 + nc));
            std::vector<double> aq(a.begin() + f0, a.begin() + f0 + nc);
            std::vector<float> f;
            nce::patch_features(fr, nc, c->eps, c->tab.problem, aq, f);
            all.insert(all.end(), f.begin(), f.end());
        }
        bt->g_feat[g].upload(all, s);
    }
}

// r = b - A x (FP64); returns per-segment ||r_s|| / ||b_s||
std::vector<double> batch_residual(nce_batch* bt, std::vector<double>& bn) {
    batch_matvec(bt, bt->d_x.p, bt->d_r.p, NCE_FP64);
    hipLaunchKernelGGL(k_sub_from, grid_for(bt->n), dim3(256), 0, bt->stream, bt->n, bt->d_b.p, bt->d_r.p);
    HIPCHK(hipGetLastError());
    std::vector<double> rn = seg_norm2(bt, bt->d_r.p);
    std::vector<double> rel(bt->B);
    for (int q = 0; q < bt->B; ++q) rel[q] = bn[q] > 0 ? std::sqrt(rn[q]) / bn[q] : 0.0;
    return rel;
}

int solve_batch(nce_batch* bt, double* results, double* coeffs, nce_info* infos) {
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = bt->stream;
    if (bt->precision == NCE_MIXED && bt->deflation) ensure_batch_deflation(bt);
    const int S = bt->B;
    const int64_t npatch = bt->n / bt->K;
    hipLaunchKernelGGL(k_init_rhs, grid_for(bt->n), dim3(256), 0, s, npatch, bt->K, bt->d_b.p, bt->d_x.p);
    HIPCHK(hipGetLastError());
    std::vector<double> bn = seg_norm2(bt, bt->d_b.p);
    for (double& v : bn) v = std::sqrt(v);
    std::vector<nce_info> inf(S);
    for (auto& f : inf) {
        f = nce_info{};
        f.rel_residual_x0 = 1.0;
    }
    std::vector<int> steps;
    std::vector<double> est;
    std::vector<char> todo(S, 1), done(S, 0);
    // configurations with one patch: no scattering, x = b
    for (int q = 0; q < S; ++q)
        if (bt->seg_off[q + 1] - bt->seg_off[q] == bt->K) todo[q] = 0;
    // one-patch configurations: x = b (their residual is then exactly zero)
    for (int q = 0; q < S; ++q)
        if (!todo[q])
            HIPCHK(hipMemcpyAsync(bt->d_x.p + bt->seg_off[q], bt->d_b.p + bt->seg_off[q], sizeof(double) * bt->K,
                                  hipMemcpyDeviceToDevice, s));
    // r = b - A x0 = b off the one-patch configurations
    HIPCHK(hipMemcpyAsync(bt->d_r.p, bt->d_b.p, sizeof(double) * bt->n, hipMemcpyDeviceToDevice, s));
    for (int q = 0; q < S; ++q)
        if (!todo[q]) HIPCHK(nce::fill(s, bt->K, 0.0, bt->d_r.p + bt->seg_off[q]));
    std::vector<double> rel(S, 1.0);
    for (int q = 0; q < S; ++q)
        if (!todo[q]) rel[q] = 0.0;
    if (bt->warm_coarse || bt->warm) {
        // x0_i = a_i m_i per member (m_i = e_0 without a network), r = b - A x0 in FP64
        batch_coarse(bt);
        if (bt->warm) batch_features(bt);
        for (size_t g = 0; g < bt->groups.size(); ++g) {
            nce_ctx* c = bt->groups[g];
            const float* m32 = bt->warm ? bt->warm->forward(s, bt->g_feat[g].p, c->N) : nullptr;
            HIPCHK(nce::rows_scale(s, c->N, bt->K, bt->g_a[g].p, m32, bt->d_x.p + bt->g_elem[g]));
        }
        for (int q = 0; q < S; ++q)
            if (!todo[q])
                HIPCHK(hipMemcpyAsync(bt->d_x.p + bt->seg_off[q], bt->d_b.p + bt->seg_off[q],
                                      sizeof(double) * bt->K, hipMemcpyDeviceToDevice, s));
        if (bt->precision == NCE_MIXED) {
            // FP32 r0 for every member; FP64 r0 only for the members whose guess
            // allows one refinement step to reach the tolerance (as the single
            // solve), with the other members' far fields masked off
            batch_matvec(bt, bt->d_x.p, bt->d_r.p, NCE_MIXED);
            hipLaunchKernelGGL(k_sub_from, grid_for(bt->n), dim3(256), 0, s, bt->n, bt->d_b.p, bt->d_r.p);
            HIPCHK(hipGetLastError());
            const std::vector<double> rn = seg_norm2(bt, bt->d_r.p);
            std::vector<int> exact(S, 0);
            int nexact = 0;
            for (int q = 0; q < S; ++q) {
                rel[q] = todo[q] ? std::sqrt(rn[q]) / bn[q] : 0.0;
                if (todo[q]) inf[q].iters_fp32 += 1;
                if (todo[q] && rel[q] <= bt->tol / 1e-5) {
                    exact[q] = 1;
                    ++nexact;
                }
            }
            if (nexact) {
                HIPCHK(hipMemcpyAsync(bt->d_active.p, exact.data(), sizeof(int) * S, hipMemcpyHostToDevice, s));
                batch_matvec(bt, bt->d_x.p, bt->d_w.p, NCE_FP64, bt->d_active.p);
                hipLaunchKernelGGL(k_sub_from, grid_for(bt->n), dim3(256), 0, s, bt->n, bt->d_b.p, bt->d_w.p);
                HIPCHK(hipGetLastError());
                for (int q = 0; q < S; ++q)
                    if (exact[q])
                        HIPCHK(hipMemcpyAsync(bt->d_r.p + bt->seg_off[q], bt->d_w.p + bt->seg_off[q],
                                              sizeof(double) * (bt->seg_off[q + 1] - bt->seg_off[q]),
                                              hipMemcpyDeviceToDevice, s));
                const std::vector<double> rn64 = seg_norm2(bt, bt->d_r.p);
                for (int q = 0; q < S; ++q)
                    if (exact[q]) {
                        rel[q] = std::sqrt(rn64[q]) / bn[q];
                        inf[q].iters_fp64 += 1;
                    }
            }
        } else {
            rel = batch_residual(bt, bn);
            for (int q = 0; q < S; ++q)
                if (todo[q]) inf[q].iters_fp64 += 1;
        }
        for (int q = 0; q < S; ++q) {
            if (!todo[q]) continue;
            inf[q].rel_residual_x0 = rel[q];
            if (!(rel[q] < 0.99)) {
                // no gain for this member: start it from zero
                inf[q].used_fallback = 1;
                HIPCHK(nce::fill(s, bt->seg_off[q + 1] - bt->seg_off[q], 0.0, bt->d_x.p + bt->seg_off[q]));
                HIPCHK(hipMemcpyAsync(bt->d_r.p + bt->seg_off[q], bt->d_b.p + bt->seg_off[q],
                                      sizeof(double) * (bt->seg_off[q + 1] - bt->seg_off[q]),
                                      hipMemcpyDeviceToDevice, s));
                rel[q] = 1.0;
            }
        }
    }
    if (bt->precision == NCE_FP64) {
        // restarted lockstep GMRES(maxit) on the residual until every configuration converges
        for (int cycle = 0; cycle < 8; ++cycle) {
            std::vector<char> mask(S, 0);
            std::vector<double> tol(S, 1.0);
            int nact = 0;
            for (int q = 0; q < S; ++q)
                if (todo[q] && rel[q] > bt->tol) {
                    mask[q] = 1;
                    tol[q] = bt->tol / rel[q];
                    ++nact;
                }
            if (nact == 0) break;
            gmres_batch(bt, bt->d_r.p, bt->d_x.p, mask, tol, NCE_FP64, steps, est);
            const std::vector<double> before = rel;
            rel = batch_residual(bt, bn);
            for (int q = 0; q < S; ++q) {
                if (!mask[q]) {
                    rel[q] = before[q];
                    continue;
                }
                inf[q].iters_fp64 += steps[q] + 1;
                inf[q].outer += 1;
            }
        }
    } else {
        // FP64 iterative refinement around lockstep FP32 GMRES
        const int max_outer = 12;
        std::vector<double> prev(S);
        for (int outer = 0; outer < max_outer; ++outer) {
            std::vector<char> mask(S, 0);
            std::vector<double> tol(S, 1.0);
            int nact = 0;
            for (int q = 0; q < S; ++q)
                if (todo[q] && rel[q] > bt->tol) {
                    mask[q] = 1;
                    tol[q] = std::max(1e-5, 0.5 * bt->tol / rel[q]);
                    ++nact;
                }
            if (nact == 0) break;
            gmres_batch(bt, bt->d_r.p, bt->d_x.p, mask, tol, NCE_MIXED, steps, est);
            prev = rel;
            rel = batch_residual(bt, bn);
            std::vector<char> stall(S, 0);
            int nstall = 0;
            for (int q = 0; q < S; ++q) {
                if (!mask[q]) {
                    rel[q] = prev[q];  // unchanged configurations keep their last verified residual
                    continue;
                }
                inf[q].iters_fp32 += steps[q];
                inf[q].iters_fp64 += 1;
                inf[q].outer += 1;
                if (rel[q] > bt->tol && !(rel[q] < 0.5 * prev[q])) {
                    stall[q] = 1;
                    ++nstall;
                }
            }
            if (nstall) {
                // refinement stalled: finish those configurations with FP64 GMRES
                std::vector<double> tol64(S, 1.0);
                for (int q = 0; q < S; ++q)
                    if (stall[q]) {
                        tol64[q] = bt->tol / rel[q];
                        inf[q].used_fallback = 1;
                    }
                gmres_batch(bt, bt->d_r.p, bt->d_x.p, stall, tol64, NCE_FP64, steps, est);
                const std::vector<double> before = rel;
                rel = batch_residual(bt, bn);
                for (int q = 0; q < S; ++q) {
                    if (stall[q]) {
                        inf[q].iters_fp64 += steps[q] + 1;
                        todo[q] = 0;
                        done[q] = 1;
                    } else {
                        rel[q] = before[q];
                    }
                }
            }
        }
    }
    // patch fluxes I . f_i, per group, then per configuration on the host
    for (size_t g = 0; g < bt->groups.size(); ++g) {
        nce_ctx* c = bt->groups[g];
        const int64_t p0 = bt->g_elem[g] / bt->K;
        HIPCHK(nce::patch_flux(s, (int)c->N, bt->K, c->d_I.p, bt->d_x.p + bt->g_elem[g], bt->d_flux.p + p0,
                               c->d_partial.p, c->d_scal.p));
    }
    std::vector<double> flux(npatch);
    HIPCHK(hipMemcpyAsync(flux.data(), bt->d_flux.p, sizeof(double) * npatch, hipMemcpyDeviceToHost, s));
    if (coeffs) HIPCHK(hipMemcpyAsync(coeffs, bt->d_x.p, sizeof(double) * bt->n, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool all = true;
    for (int q = 0; q < S; ++q) {
        double Is = 0.0;
        for (int64_t i = bt->seg_off[q] / bt->K; i < bt->seg_off[q + 1] / bt->K; ++i) Is += flux[i];
        const int b = bt->seg_cfg[q];
        const int prob = bt->g_problem[bt->seg_group[q]];
        results[b] = prob == NCE_INTERIOR ? 1.0 / (3.0 * Is) - 0.6 : 4.0 * M_PI * Is;
        inf[q].rel_residual = rel[q];
        inf[q].t_solve_s = t;
        if (!(rel[q] <= bt->tol * 1.0001)) all = false;
        if (infos) infos[b] = inf[q];
    }
    return all ? NCE_OK : NCE_NOTCONVERGED;
}

}  // namespace

extern "C" {

int nce_setup_batch(const double* const* centers, const int64_t* N, const double* eps, const int* problem, int B,
                    const nce_opts* opts_in, nce_batch** out) {
    g_err.clear();
    if (!out) return fail(NCE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!centers || !N || !eps || !problem || B < 1) return fail(NCE_EINVAL, "need B >= 1 configurations");
    nce_opts o;
    nce_default_opts(&o);
    if (opts_in) o = *opts_in;
    if (o.max_iter > kMaxBatchIter) return fail(NCE_EINVAL, "max_iter of a batch must not exceed 120");
    // groups by (problem, eps)
    std::map<std::pair<int, double>, std::vector<int>> groups;
    for (int b = 0; b < B; ++b) {
        if (!centers[b] || N[b] < 1) return fail(NCE_EINVAL, "configuration " + std::to_string(b) + ": need N >= 1");
        nce_opts ob = o;
        ob.problem = problem[b];
        int rc = validate_opts(ob, eps[b]);
        if (rc != NCE_OK) {
            g_err = "configuration " + std::to_string(b) + ": " + g_err;
            return rc;
        }
        const std::vector<int64_t> one{0, N[b]};
        rc = validate_centers(centers[b], one, eps[b]);
        if (rc != NCE_OK) {
            g_err = "configuration " + std::to_string(b) + ": " + g_err;
            return rc;
        }
        groups[{problem[b], eps[b]}].push_back(b);
    }
    return guarded([&]() -> int {
        auto* bt = new nce_batch();
        std::unique_ptr<nce_batch, void (*)(nce_batch*)> guard(bt, nce_destroy_batch);
        bt->B = B;
        if (o.stream) {
            bt->stream = (hipStream_t)o.stream;
        } else {
            HIPCHK(hipStreamCreateWithFlags(&bt->stream, hipStreamNonBlocking));
            bt->own_stream = true;
        }
        bt->cfg_seg.assign(B, -1);
        bt->g_elem = {0};
        bt->seg_off = {0};
        for (const auto& kv : groups) {
            const std::vector<int>& members = kv.second;
            std::vector<int64_t> first{0};
            std::vector<double> c;
            for (int b : members) {
                c.insert(c.end(), centers[b], centers[b] + 3 * N[b]);
                first.push_back(first.back() + N[b]);
            }
            nce_opts og = o;
            og.problem = kv.first.first;
            og.stream = bt->stream;
            auto* ctx = new nce_ctx();
            bt->groups.push_back(ctx);
            init_ctx(ctx, c.data(), first, kv.first.second, og, true);
            bt->K = ctx->K;
            const int gidx = (int)bt->groups.size() - 1;
            bt->g_problem.push_back(og.problem);
            bt->g_seg0.push_back((int)bt->seg_cfg.size());
            bt->g_elem.push_back(bt->g_elem.back() + ctx->N * ctx->K);
            for (int b : members) {
                bt->cfg_seg[b] = (int)bt->seg_cfg.size();
                bt->seg_cfg.push_back(b);
                bt->seg_group.push_back(gidx);
                bt->seg_off.push_back(bt->seg_off.back() + N[b] * (int64_t)ctx->K);
            }
        }
        bt->n = bt->seg_off.back();
        // reduction chunks: each configuration's range cut into pieces of <= kChunk
        std::vector<int64_t> ch_e0;
        std::vector<int> ch_seg, seg_ch{0};
        for (int q = 0; q < B; ++q) {
            for (int64_t e = bt->seg_off[q]; e < bt->seg_off[q + 1]; e += kChunk) {
                ch_e0.push_back(e);
                ch_seg.push_back(q);
            }
            seg_ch.push_back((int)ch_e0.size());
        }
        ch_e0.push_back(bt->n);
        bt->nch = (int)ch_seg.size();
        bt->d_ch_e0.upload(ch_e0, bt->stream);
        bt->d_ch_seg.upload(ch_seg, bt->stream);
        bt->d_seg_ch.upload(seg_ch, bt->stream);
        bt->d_xin.alloc(bt->n);
        bt->d_w.alloc(bt->n);
        bt->d_b.alloc(bt->n);
        bt->d_r.alloc(bt->n);
        bt->d_x.alloc(bt->n);
        bt->d_flux.alloc(bt->n / bt->K);
        bt->tol = o.tol_gmres;
        bt->precision = o.precision;
        bt->deflation = o.deflation != 0;
        ensure_solver(bt, o.max_iter);
        HIPCHK(hipStreamSynchronize(bt->stream));
        *out = guard.release();
        return NCE_OK;
    });
}

void nce_destroy_batch(nce_batch* bt) {
    if (!bt) return;
    if (bt->stream) (void)hipStreamSynchronize(bt->stream);
    delete bt;
}

int nce_batch_dims(const nce_batch* bt, int64_t* n_total, int* K, int* ngroups) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (n_total) *n_total = bt->n;
    if (K) *K = bt->K;
    if (ngroups) *ngroups = (int)bt->groups.size();
    return NCE_OK;
}

int nce_batch_offsets(const nce_batch* bt, int64_t* off, int* far_tree) {
    if (!bt || !off) return fail(NCE_EINVAL, "NULL argument");
    for (int b = 0; b < bt->B; ++b) {
        const int q = bt->cfg_seg[b];
        off[b] = bt->seg_off[q];
        if (far_tree) {
            const nce_ctx* g = bt->groups[bt->seg_group[q]];
            // position of configuration b inside its group
            int local = 0;
            for (int r = 0; r < q; ++r)
                if (bt->seg_group[r] == bt->seg_group[q]) ++local;
            far_tree[b] = g->cfg_tree[local];
        }
    }
    return NCE_OK;
}

int nce_batch_work(const nce_batch* bt, int precision, double* far, double* near, double* interp) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    double f = 0, nr = 0, it = 0;
    for (const nce_ctx* g : bt->groups) {
        const nce::Tree& t = (precision == NCE_MIXED && g->has_tree32) ? g->tree32 : g->tree;
        f += t.pairs_far;
        nr += t.pairs_near;
        it += t.interp_fma;
    }
    if (far) *far = f;
    if (near) *near = nr;
    if (interp) *interp = it;
    return NCE_OK;
}

int nce_batch_matvec(nce_batch* bt, const double* x, double* y, int precision) {
    if (!bt || !x || !y) return fail(NCE_EINVAL, "NULL argument");
    if (x == y) return fail(NCE_EINVAL, "x and y may not alias");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        batch_matvec(bt, x, y, precision);
        return NCE_OK;
    });
}

int nce_batch_set_solver(nce_batch* bt, double tol, int max_iter, int precision, int use_graph) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (!(tol > 0 && tol < 1)) return fail(NCE_EINVAL, "tol_gmres must lie in (0, 1)");
    if (max_iter < 1 || max_iter > kMaxBatchIter) return fail(NCE_EINVAL, "max_iter must lie in [1, 120]");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        if (max_iter != bt->maxit) {
            HIPCHK(hipStreamSynchronize(bt->stream));
            bt->maxit = 0;
            ensure_solver(bt, max_iter);
        }
        bt->tol = tol;
        bt->precision = precision;
        bt->use_graph = use_graph ? 1 : 0;
        return NCE_OK;
    });
}

int nce_batch_autotune(nce_batch* bt, int precision, int* choice) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (precision != NCE_FP64 && precision != NCE_MIXED) return fail(NCE_EINVAL, "bad precision");
    return guarded([&]() -> int {
        const int ti = precision == NCE_FP64 ? 0 : 1;
        for (size_t g = 0; g < bt->groups.size(); ++g) {
            autotune(bt->groups[g], precision);
            if (choice) {
                choice[2 * g] = bt->groups[g]->tune_p2l[ti];
                choice[2 * g + 1] = bt->groups[g]->tune_l2t[ti];
            }
        }
        // captured steps hold the old kernel shapes
        if (bt->graph[ti]) {
            (void)hipGraphExecDestroy(bt->graph[ti]);
            bt->graph[ti] = nullptr;
        }
        return NCE_OK;
    });
}

int nce_batch_set_warm_start(nce_batch* bt, nce_mlp* m, int use_coarse) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (m && (m->net.n_in != nce::kFeatureDim || m->net.n_out != bt->K))
        return fail(NCE_ESTATE, "network shape does not match NCE_FEATURES -> K");
    if (m && !use_coarse) return fail(NCE_EINVAL, "the network refines the coarse solve: use_coarse must be 1");
    return guarded([&]() -> int {
        bt->warm = m ? &m->net : nullptr;
        bt->warm_coarse = use_coarse != 0;
        // per-layout preprocessing now, not inside the next solve
        if (bt->warm_coarse) batch_coarse(bt);
        if (bt->warm) batch_features(bt);
        return NCE_OK;
    });
}

int nce_batch_set_deflation(nce_batch* bt, int on) {
    if (!bt) return fail(NCE_EINVAL, "batch is NULL");
    if (on != 0 && on != 1) return fail(NCE_EINVAL, "on must be 0 or 1");
    return guarded([&]() -> int {
        if (bt->deflation != (on == 1)) drop_graphs(bt);  // the captured step differs
        bt->deflation = on == 1;
        if (bt->deflation && bt->precision == NCE_MIXED) ensure_batch_deflation(bt);
        return NCE_OK;
    });
}

int nce_solve_batch(nce_batch* bt, double* results, double* coeffs, nce_info* infos) {
    if (!bt || !results) return fail(NCE_EINVAL, "NULL argument");
    return guarded([&]() -> int { return solve_batch(bt, results, coeffs, infos); });
}

}  // extern "C"
