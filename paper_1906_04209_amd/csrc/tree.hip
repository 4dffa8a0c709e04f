// Device side of the hierarchical far field: P2L onto incoming grids,
// per-grid reduction and Chebyshev-Fourier transform, direct-list sums, and
// interpolation at the sampling nodes (Section 8, Step 3 items 2-4). gfx950.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>

#include <stdexcept>
#include <string>

#include "greens.hpp"
#include "kernels.hpp"
#include "tree.hpp"

namespace nce {

namespace {

constexpr double kPi = 3.14159265358979323846;

// grid point t = a * nt + b of a grid with nr radial Chebyshev nodes on
// [0, 1] (positive half of the 2 nr first-kind nodes on [-1, 1]) and nt
// angles, in the stereographic polar coordinates of its cap: the node x sits
// at u = Tc x, u = tan(phi / 2) for a point at arclength phi from the cap
// centre, Tc = tan(R / 2) for the cap radius R. Returns the point's local
// offset (cos phi - 1, sin phi cos th, sin phi sin th).
__device__ __forceinline__ void grid_point(int t, int nr, int nt, double Tc, double& o0, double& o1, double& o2) {
    const int a = t / nt, b = t - a * nt;
    const double u = Tc * cospi((2.0 * a + 1.0) / (4.0 * nr));
    double sb, cb;
    sincospi(2.0 * b / nt, &sb, &cb);
    const double d = 1.0 / (1.0 + u * u);
    o0 = -2.0 * u * u * d;
    const double s = 2.0 * u * d;
    o1 = s * cb;
    o2 = s * sb;
}

// Half-scaled grid points of every grid, relative to its cap centre, in the
// global frame (FP64 and FP32 copies); one block per grid, once per tree.
__global__ __launch_bounds__(256) void k_grid_points(const int* __restrict__ g_nr, const int* __restrict__ g_nt,
                                                     const double* __restrict__ g_T, const double* __restrict__ g_frame,
                                                     const int64_t* __restrict__ g_off, double* __restrict__ out64,
                                                     float* __restrict__ out32) {
    const int g = blockIdx.x;
    const int nr = g_nr[g], nt = g_nt[g], q = nr * nt;
    const double* fg = g_frame + 9 * (int64_t)g;
    for (int t = threadIdx.x; t < q; t += blockDim.x) {
        double o0, o1, o2;
        grid_point(t, nr, nt, g_T[g], o0, o1, o2);
        const int64_t e = 3 * (g_off[g] + t);
        for (int c = 0; c < 3; ++c) {
            const double v = 0.5 * (o0 * fg[c] + o1 * fg[3 + c] + o2 * fg[6 + c]);
            out64[e + c] = v;
            out32[e + c] = (float)v;
        }
    }
}

// ---------------------------------------------------- reduce + transform
// A grid's q values sv (LDS, doubles) to its Chebyshev-Fourier coefficients:
// the angular DFT and the parity-restricted radial Chebyshev transform.
// Coefficient layout: mode m = 0..nt-1 (m <= nt/2: cos(m th); m > nt/2:
// sin((m - nt/2) th)), radial index n' (Chebyshev degree 2 n' + parity of the
// angular order). sa: LDS scratch of q doubles; tc, ts (nt) and tch (8 nr):
// LDS tables, contiguous (ts = tc + nt, tch = tc + 2 nt). Every thread of the
// block calls it after sv is complete.
template <class T, class TT>
__device__ void grid_transform(const double* sv, double* sa, TT* tc, TT* ts, TT* tch, int nr, int nt,
                               const double* __restrict__ gtab, T* __restrict__ coef) {
    const int q = nr * nt;
    // trigonometric tables (gtab, per (nr, nt), from the host): cos, sin(2 pi
    // j / nt) and cos(2 pi j / (8 nr)), contiguous as tc, ts, tch
    for (int j = threadIdx.x; j < 2 * nt + 8 * nr; j += blockDim.x) tc[j] = (TT)gtab[j];
    __syncthreads();
    const int half = nt / 2;
    // angular transform: sa[m * nr + a]
    for (int idx = threadIdx.x; idx < q; idx += blockDim.x) {
        const int m = idx / nr, a = idx - m * nr;
        const bool is_sin = m > half;
        const int k = is_sin ? m - half : m;
        const double wgt = (k == 0 || k == half) ? 1.0 / nt : 2.0 / nt;
        double acc = 0.0;
        int red = 0;
        for (int b = 0; b < nt; ++b) {
            acc += sv[a * nt + b] * (double)(is_sin ? ts[red] : tc[red]);
            red += k;
            if (red >= nt) red -= nt;
        }
        sa[idx] = wgt * acc;
    }
    __syncthreads();
    // radial transform on the positive first-kind Chebyshev nodes (parity):
    // T_n(x_a) = cos(2 pi n (2a+1) / (8 nr))
    for (int idx = threadIdx.x; idx < q; idx += blockDim.x) {
        const int m = idx / nr, np = idx - m * nr;
        const int k = m > half ? m - half : m;
        const int n = 2 * np + (k & 1);
        double acc = 0.0;
        for (int a = 0; a < nr; ++a) acc += sa[m * nr + a] * (double)tch[(n * (2 * a + 1)) % (8 * nr)];
        coef[idx] = (T)((n == 0 ? 1.0 : 2.0) / nr * acc);
    }
}

// The end of a P2L block: the group partial sums red[sp q + t] (sp < ns) of
// the item. An item that is its grid's only one (solo) sums them and turns
// them into the grid's coefficients itself, in the staging LDS (sv, sa in
// `big`, at least 2 kMaxGridQ doubles; the tables in `tab`, at least 2
// kMaxGridNt + 8 kMaxGridNr values); any other writes its partial sums for
// k_reduce_coef. Every thread of the block calls it after red is complete.
template <class T, class TT>
__device__ __forceinline__ void p2l_finish(const double* red, int ns, int q, bool solo, int nr, int nt,
                                           double* big, TT* tab, const double* __restrict__ gtab,
                                           T* __restrict__ part, T* __restrict__ coef) {
    if (!solo) {
        for (int t = threadIdx.x; t < q; t += blockDim.x) {
            double v = 0.0;
            for (int sp = 0; sp < ns; ++sp) v += red[sp * q + t];
            part[t] = (T)v;
        }
        return;
    }
    constexpr int kPer = kMaxGridQ / 256;
    double v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int t = threadIdx.x + k * 256;
        v[k] = 0.0;
        if (t < q)
            for (int sp = 0; sp < ns; ++sp) v[k] += red[sp * q + t];
    }
    __syncthreads();  // red (which may share `big`) is consumed
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
        const int t = threadIdx.x + k * 256;
        if (t < q) big[t] = v[k];
    }
    __syncthreads();
    grid_transform<T, TT>(big, big + q, tab, tab + nt, tab + 2 * nt, nr, nt, gtab, coef);
}

// One block per grid of `glist` (the grids with more than one P2L item, or
// every grid when glist is null): sum the items' partial sums in item order,
// then the transform.
template <class T>
__global__ __launch_bounds__(256) void k_reduce_coef(const int* __restrict__ glist, const int* __restrict__ g_nr,
                                                     const int* __restrict__ g_nt, const int64_t* __restrict__ g_off,
                                                     const int* __restrict__ g_item0, const int* __restrict__ g_item1,
                                                     const int64_t* __restrict__ it_off, const T* __restrict__ part,
                                                     T* __restrict__ coef, const int* __restrict__ g_cfg,
                                                     const int* __restrict__ live, const double* __restrict__ ttab,
                                                     const int* __restrict__ g_ttab) {
    __shared__ double sv[kMaxGridQ];
    __shared__ double sa[kMaxGridQ];
    __shared__ T tab[2 * kMaxGridNt + 8 * kMaxGridNr];
    const int g = glist ? glist[blockIdx.x] : (int)blockIdx.x;
    if (live && !live[g_cfg[g]]) return;
    const int nr = g_nr[g], nt = g_nt[g], q = nr * nt;
    const int i0 = g_item0[g], i1 = g_item1[g];
    for (int t = threadIdx.x; t < q; t += blockDim.x) {
        double acc = 0.0;
        for (int it = i0; it < i1; ++it) acc += (double)part[it_off[it] + t];
        sv[t] = acc;
    }
    __syncthreads();
    grid_transform<T, T>(sv, sa, tab, tab + nt, tab + 2 * nt, nr, nt, ttab + g_ttab[g], coef + g_off[g]);
}

// ----------------------------------------------------------------- P2L
// One block per work item (one grid and a run of its source patches). The
// 256 threads are split into ns groups; each thread owns up to R grid points
// (spaced qq = ceil(q/R) apart; R = 4 or 8, chosen by the autotuner) and takes
// every ns-th staged source point, so small grids still keep every lane busy.
// The item's source skeleton points (of the outgoing table its grid uses) and
// strengths are staged in LDS in batches of kStage points, positions relative
// to the grid's cap centre; every batch is padded with ns points of zero
// strength so that all groups run the same number of iterations (loop control
// on the scalar unit). The groups' partial sums are combined in LDS and
// written per item to `part`.
constexpr int kStage = 1024;
constexpr int kStage64 = 448;  // FP64: 40 bytes per staged point (with the 32 KiB logarithm window, 3 blocks per CU)
constexpr int kStagePad = 64;  // >= the largest ns

// floor(a / b) for 0 <= a < 2^21, 1 <= b < 2^12, by one reciprocal: the
// quotient's fractional part is at least 0.5 / b away from the next integer,
// far more than the reciprocal's error
__device__ __forceinline__ int div_small(int a, float inv_b) { return (int)(((float)a + 0.5f) * inv_b); }

// An item's sources by outgoing table (the tree sorts a grid's sources by
// table, so they form at most kMaxTableRuns runs): run k stages the points
// [pt0[k], pt0[k + 1]) of the item, sources src[s0[k] ..] with skeleton size
// p[k], first skeleton offset toff[k] and strength column col[k].
struct StageRuns {
    int n;
    int pt0[kMaxTableRuns + 1];
    int s0[kMaxTableRuns], p[kMaxTableRuns], toff[kMaxTableRuns], col[kMaxTableRuns];
    float inv[kMaxTableRuns];
};

// Fills sr for `item` (tb0: the first table index of the item's source type);
// every thread of the block calls it. Returns the item's staged point count.
__device__ __forceinline__ int load_runs(StageRuns& sr, const TabRuns& tr, int item, int src_end, int tb0,
                                         const int* __restrict__ t_off, const int* __restrict__ t_col,
                                         const int* __restrict__ t_p) {
    const int r0 = tr.it_run0[item], nr = tr.it_run0[item + 1] - r0;
    const int k = threadIdx.x;
    if (k < nr) {
        const int s = tr.run_src[r0 + k], e = k + 1 < nr ? tr.run_src[r0 + k + 1] : src_end;
        const int tb = tb0 + tr.run_tab[r0 + k], pk = t_p[tb];
        sr.s0[k] = s;
        sr.p[k] = pk;
        sr.toff[k] = t_off[tb];
        sr.col[k] = t_col ? t_col[tb] : t_off[tb];
        sr.inv[k] = __builtin_amdgcn_rcpf((float)pk);
        sr.pt0[k + 1] = (e - s) * pk;   // the run's points, summed below
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sr.n = nr;
        sr.pt0[0] = 0;
        for (int j = 1; j <= nr; ++j) sr.pt0[j] += sr.pt0[j - 1];
    }
    __syncthreads();
    return sr.pt0[nr];
}

// Staged point e of the item: its source's place in the source list, its
// skeleton point's offset index and its strength column.
__device__ __forceinline__ void run_point(const StageRuns& sr, int e, int& sidx, int& oidx, int& cidx) {
    int k = 0;
    while (k + 1 < sr.n && e >= sr.pt0[k + 1]) ++k;
    const int el = e - sr.pt0[k], js = div_small(el, sr.inv[k]), m = el - js * sr.p[k];
    sidx = sr.s0[k] + js;
    oidx = sr.toff[k] + m;
    cidx = sr.col[k] + m;
}

template <int R>
__device__ __forceinline__ void p2l_layout(int q, int& qq, int& ns, int& split, int& t0) {
    qq = (q + R - 1) / R;
    const float inv = __builtin_amdgcn_rcpf((float)qq);
    ns = div_small(256, inv);
    ns = ns < 1 ? 1 : (ns > kStagePad ? kStagePad : ns);
    split = div_small((int)threadIdx.x, inv);
    t0 = threadIdx.x - split * qq;
}

template <int PROB, int R>
__global__ __launch_bounds__(256) void k_p2l64(const int* __restrict__ it_grid, const int* __restrict__ it_src0,
                                               const int* __restrict__ it_src1, const int64_t* __restrict__ it_off,
                                               const int* __restrict__ src, const double* __restrict__ g_frame,
                                               const double* __restrict__ g_T, const int* __restrict__ g_nr,
                                               const int* __restrict__ g_nt, TabRuns tr,
                                               const int* __restrict__ t_off, const int* __restrict__ t_p,
                                               const double* __restrict__ frames, const double* __restrict__ skel_off,
                                               const double* __restrict__ rho, int ptot, double* __restrict__ part,
                                               const int* __restrict__ it_type, const int* __restrict__ t_col,
                                               int ntab,
                                               const int* __restrict__ it_cfg, const int* __restrict__ live,
                                               const int64_t* __restrict__ g_off, const double* __restrict__ gpt,
                                               const int* __restrict__ it_list, const int* __restrict__ it_win,
                                               const LogEntry* __restrict__ logwin, int win_first,
                                               const int* __restrict__ it_solo, double* __restrict__ coef,
                                               const double* __restrict__ ttab, const int* __restrict__ g_ttab) {
    // staging (kStage64 points: (-2 a, |a|^2) with a the quarter-scaled
    // offset from the cap centre, and the strengths) and, after the sums, the split
    // partials (ns q <= 256 R); the item's logarithm window, and after the
    // sums the transform's tables
    __shared__ double4 smem4[kStage64 + kStagePad];
    __shared__ double srho[kStage64 + kStagePad];
    __shared__ LogEntry ltab[kWinTab];
    static_assert((kStage64 + kStagePad) * 4 >= 2 * kMaxGridQ, "split partials and the grid transform's values");
    static_assert(kWinTab * 2 >= 2 * kMaxGridNt + 8 * kMaxGridNr, "the grid transform's tables");
    double* smem = reinterpret_cast<double*>(smem4);
    const int item = it_list ? it_list[blockIdx.x] : (int)blockIdx.x;
    if (live && !live[it_cfg[item]]) return;
    {
        // slot s of the window holds octave window_octave(e0, s), one of the
        // kWinOct octaves from e0 on (all inside the table by construction)
        const int e0 = it_win[item];
        for (int k = threadIdx.x; k < kWinTab; k += blockDim.x)
            ltab[k] = logwin[(window_octave(e0, k >> kWinBinBits) - win_first) * kWinBins + (k & (kWinBins - 1))];
    }
    const int g = it_grid[item];
    const int nr = g_nr[g], nt = g_nt[g], q = nr * nt;
    // outgoing table: the grid's, of the item's source type with several radii
    __shared__ StageRuns sruns;
    const int total = load_runs(sruns, tr, item, it_src1[item], it_type ? it_type[item] * ntab : 0, t_off, t_col, t_p);
    const double* fg = g_frame + 9 * (int64_t)g;
    int qq, ns, split, t0;
    p2l_layout<R>(q, qq, ns, split, t0);
    const bool active = split < ns;
    double zx[R], zy[R], zz[R], z2[R], acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = t0 + r * qq;
        acc[r] = 0.0;
        zx[r] = zy[r] = zz[r] = 0.0;
        if (active && t < q) {
            // quarter-scaled offsets from the cap centre (the tree stores them
            // half-scaled; the extra factor 1/2 is exact)
            const double* z = gpt + 3 * (g_off[g] + t);
            zx[r] = 0.5 * z[0];
            zy[r] = 0.5 * z[1];
            zz[r] = 0.5 * z[2];
        }
        z2[r] = zx[r] * zx[r] + zy[r] * zy[r] + zz[r] * zz[r];
    }
    for (int c0 = 0; c0 < total; c0 += kStage64) {
        const int cl = min(kStage64, total - c0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cl + ns; idx += blockDim.x) {
            double ax = 8.0, ay = 8.0, az = 8.0, w = 0.0;  // padding: far away, zero strength
            if (idx < cl) {
                int sidx, oidx, cidx;
                run_point(sruns, c0 + idx, sidx, oidx, cidx);
                const int j = src[sidx];
                const double* fj = frames + 9 * (int64_t)j;
                const double* o = skel_off + 3 * (int64_t)oidx;
                ax = 0.25 * ((fj[0] - fg[0]) + (o[0] * fj[0] + o[1] * fj[3] + o[2] * fj[6]));
                ay = 0.25 * ((fj[1] - fg[1]) + (o[0] * fj[1] + o[1] * fj[4] + o[2] * fj[7]));
                az = 0.25 * ((fj[2] - fg[2]) + (o[0] * fj[2] + o[1] * fj[5] + o[2] * fj[8]));
                w = rho[(int64_t)j * ptot + cidx];
            }
            // |z - a|^2 = |z|^2 + |a|^2 - 2 z.a: grid points lie within the cap
            // and sources at least a cap radius beyond it, so the cancellation
            // costs at most a factor 5 in relative rounding
            smem4[idx] = make_double4(-2.0 * ax, -2.0 * ay, -2.0 * az, ax * ax + ay * ay + az * az);
            srho[idx] = w;
        }
        __syncthreads();
        // the same trip count for every group: points cl .. cl + ns - 1 are padding
        const int nit = (cl + ns - 1) / ns;
        if (active) {
            const double4* a_ptr = smem4 + split;
            const double* w_ptr = srho + split;
            // two points per pass: the second reads are in flight while the
            // first point is summed
#pragma unroll 2
            for (int it = 0; it < nit; ++it, a_ptr += ns, w_ptr += ns) {
                const double4 a = *a_ptr;
                const double w = *w_ptr;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // s = d^2 / 16
                    const double s = fma(zx[r], a.x, fma(zy[r], a.y, fma(zz[r], a.z, a.w))) + z2[r];
                    acc[r] = fma(green64_grid_win<PROB>(s, ltab), w, acc[r]);
                }
            }
        }
    }
    __syncthreads();
    double* red = smem;  // ns * q <= 256 R partial sums
    if (active)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = t0 + r * qq;
            if (t < q) red[split * q + t] = acc[r];
        }
    __syncthreads();
    p2l_finish<double, double>(red, ns, q, it_solo && it_solo[item], nr, nt, smem, reinterpret_cast<double*>(ltab),
                               ttab + g_ttab[g], part + it_off[item], coef + g_off[g]);
}

template <int PROB, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(R == 4 ? 7 : 1))) void k_p2l32(const int* __restrict__ it_grid, const int* __restrict__ it_src0,
                                               const int* __restrict__ it_src1, const int64_t* __restrict__ it_off,
                                               const int* __restrict__ src, const double* __restrict__ g_frame,
                                               const double* __restrict__ g_T, const int* __restrict__ g_nr,
                                               const int* __restrict__ g_nt, TabRuns tr,
                                               const int* __restrict__ t_off, const int* __restrict__ t_p,
                                               const double* __restrict__ frames, const float* __restrict__ skel_off,
                                               const float* __restrict__ rho, int ptot, float* __restrict__ part,
                                               const int* __restrict__ it_type, const int* __restrict__ t_col,
                                               int ntab,
                                               const int* __restrict__ it_cfg, const int* __restrict__ live,
                                               const int64_t* __restrict__ g_off, const float* __restrict__ gpt,
                                               const int* __restrict__ it_list,
                                               const int* __restrict__ it_solo, float* __restrict__ coef,
                                               const double* __restrict__ ttab, const int* __restrict__ g_ttab) {
    // staging (kStage points: (-2 a, |a|^2) with a the half-scaled offset from
    // the cap centre, and the strengths) and, after the sums, the split
    // partials (ns q <= 256 R doubles, in smem4)
    __shared__ float4 smem4[kStage + kStagePad];
    __shared__ float srho[kStage + kStagePad];
    double* smem = reinterpret_cast<double*>(smem4);
    const int item = it_list ? it_list[blockIdx.x] : (int)blockIdx.x;
    if (live && !live[it_cfg[item]]) return;
    const int g = it_grid[item];
    const int nr = g_nr[g], nt = g_nt[g], q = nr * nt;
    // outgoing table: the grid's, of the item's source type with several radii
    __shared__ StageRuns sruns;
    const int total = load_runs(sruns, tr, item, it_src1[item], it_type ? it_type[item] * ntab : 0, t_off, t_col, t_p);
    const double* fg = g_frame + 9 * (int64_t)g;
    int qq, ns, split, t0;
    p2l_layout<R>(q, qq, ns, split, t0);
    const bool active = split < ns;
    float zx[R], zy[R], zz[R], z2[R];
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int t = t0 + r * qq;
        acc[r] = 0.0;
        zx[r] = zy[r] = zz[r] = 0.0f;
        if (active && t < q) {
            // half-scaled offsets from the cap centre, precomputed per tree
            const float* z = gpt + 3 * (g_off[g] + t);
            zx[r] = z[0];
            zy[r] = z[1];
            zz[r] = z[2];
        }
        z2[r] = zx[r] * zx[r] + zy[r] * zy[r] + zz[r] * zz[r];
    }
    constexpr float kLn2 = 0.69314718055994530942f;
    for (int c0 = 0; c0 < total; c0 += kStage) {
        const int cl = min(kStage, total - c0);
        __syncthreads();
        for (int idx = threadIdx.x; idx < cl + ns; idx += blockDim.x) {
            float ax = 8.0f, ay = 8.0f, az = 8.0f, w = 0.0f;  // padding: far away, zero strength
            if (idx < cl) {
                int sidx, oidx, cidx;
                run_point(sruns, c0 + idx, sidx, oidx, cidx);
                const int j = src[sidx];
                const double* fj = frames + 9 * (int64_t)j;
                const float* o = skel_off + 3 * (int64_t)oidx;
                ax = 0.5f * ((float)(fj[0] - fg[0]) + (o[0] * (float)fj[0] + o[1] * (float)fj[3] + o[2] * (float)fj[6]));
                ay = 0.5f * ((float)(fj[1] - fg[1]) + (o[0] * (float)fj[1] + o[1] * (float)fj[4] + o[2] * (float)fj[7]));
                az = 0.5f * ((float)(fj[2] - fg[2]) + (o[0] * (float)fj[2] + o[1] * (float)fj[5] + o[2] * (float)fj[8]));
                w = rho[(int64_t)j * ptot + cidx];
            }
            // |z - a|^2 = |z|^2 + |a|^2 - 2 z.a (cancellation at most a factor 5,
            // as in the FP64 kernel)
            smem4[idx] = make_float4(-2.0f * ax, -2.0f * ay, -2.0f * az, ax * ax + ay * ay + az * az);
            srho[idx] = w;
        }
        __syncthreads();
        // the same trip count for every group: points cl .. cl + ns - 1 are padding
        const int nit = (cl + ns - 1) / ns;
        if (active) {
            // FP32 sums over at most 256 points, carried in FP64 between runs
            const float4* a_ptr = smem4 + split;
            const float* w_ptr = srho + split;
            for (int i0 = 0; i0 < nit; i0 += 256) {
                const int i1 = min(nit, i0 + 256);
                float aw[R], al[R];
#pragma unroll
                for (int r = 0; r < R; ++r) aw[r] = al[r] = 0.0f;
                for (int it = i0; it < i1; ++it, a_ptr += ns, w_ptr += ns) {
                    const float4 a = *a_ptr;
                    const float sw = *w_ptr;
#pragma unroll
                    for (int r = 0; r < R; ++r) {
                        const float h2 = fmaf(zx[r], a.x, fmaf(zy[r], a.y, fmaf(zz[r], a.z, a.w))) + z2[r];
                        float w, l2;
                        green32_parts_half<PROB>(h2, w, l2);
                        aw[r] += w * sw;
                        al[r] += l2 * sw;
                    }
                }
#pragma unroll
                for (int r = 0; r < R; ++r) acc[r] += (double)(aw[r] - kLn2 * al[r]);
            }
        }
    }
    __syncthreads();
    double* red = smem;
    if (active)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int t = t0 + r * qq;
            if (t < q) red[split * q + t] = acc[r];
        }
    __syncthreads();
    p2l_finish<float, float>(red, ns, q, it_solo && it_solo[item], nr, nt, smem, srho, ttab + g_ttab[g],
                             part + it_off[item], coef + g_off[g]);
}

// ------------------------------------------------- P2L on the matrix cores
// The squared half-distances of a 16 x 16 tile of (grid point, source point)
// pairs are one 16 x 16 x 4 product, h2 = |z|^2 + [z, 1] . [-2 a, |a|^2], which
// the matrix cores compute (v_mfma_*_16x16x4) while the vector units evaluate
// G on the previous tile: per pair the VALU keeps the reciprocal square root,
// the logarithm and the accumulation, and the four distance multiply-adds
// move to the MFMA pipe. Wave w takes the 16-point row tiles w, w + 4, ...
// of the grid; each lane ends a tile with 4 pairs' G for one source column and
// its 4 rows, and the 16 columns are summed across lanes at the end of every
// staged batch into a per-grid-point LDS partial. Staging (positions relative
// to the cap centre, padded with zero-strength points far away) as in k_p2l64.
typedef double v4d_t __attribute__((ext_vector_type(4)));
typedef float v4f_t __attribute__((ext_vector_type(4)));
constexpr int kStageM = 640;  // staged source points per batch (multiple of 16)

template <int PROB>
__global__ __launch_bounds__(256) void k_p2l64_mfma(const int* __restrict__ it_grid, const int* __restrict__ it_src0,
                                                    const int* __restrict__ it_src1, const int64_t* __restrict__ it_off,
                                                    const int* __restrict__ src, const double* __restrict__ g_frame,
                                                    const int* __restrict__ g_nr, const int* __restrict__ g_nt,
                                                    TabRuns tr, const int* __restrict__ t_off,
                                                    const int* __restrict__ t_p, const double* __restrict__ frames,
                                                    const double* __restrict__ skel_off, const double* __restrict__ rho,
                                                    int ptot, double* __restrict__ part,
                                                    const int* __restrict__ it_type, const int* __restrict__ t_col,
                                                    int ntab, const int* __restrict__ it_cfg,
                                                    const int* __restrict__ live, const int64_t* __restrict__ g_off,
                                                    const double* __restrict__ gpt, const int* __restrict__ it_list,
                                                    const LogEntry* __restrict__ logtab) {
    __shared__ double4 smem4[kStageM];
    __shared__ double srho[kStageM];
    __shared__ double red[kMaxGridQ];
    __shared__ LogEntry ltab[kLogTab];
    const int item = it_list ? it_list[blockIdx.x] : (int)blockIdx.x;
    if (live && !live[it_cfg[item]]) return;
    for (int k = threadIdx.x; k < kLogTab; k += blockDim.x) ltab[k] = logtab[k];
    const int g = it_grid[item];
    const int q = g_nr[g] * g_nt[g];
    __shared__ StageRuns sruns;
    const int total = load_runs(sruns, tr, item, it_src1[item], it_type ? it_type[item] * ntab : 0, t_off, t_col, t_p);
    const double* fg = g_frame + 9 * (int64_t)g;
    const double* zg = gpt + 3 * g_off[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = lane & 15, kq = lane >> 4;
    const int nrt = (q + 15) >> 4;
    for (int t = threadIdx.x; t < q; t += blockDim.x) red[t] = 0.0;
    for (int c0 = 0; c0 < total; c0 += kStageM) {
        const int cl = min(kStageM, total - c0);
        const int cl16 = (cl + 15) & ~15;
        __syncthreads();
        for (int idx = threadIdx.x; idx < cl16; idx += blockDim.x) {
            double ax = 8.0, ay = 8.0, az = 8.0, w = 0.0;  // padding: far away, zero strength
            if (idx < cl) {
                int sidx, oidx, cidx;
                run_point(sruns, c0 + idx, sidx, oidx, cidx);
                const int j = src[sidx];
                const double* fj = frames + 9 * (int64_t)j;
                const double* o = skel_off + 3 * (int64_t)oidx;
                ax = 0.5 * ((fj[0] - fg[0]) + (o[0] * fj[0] + o[1] * fj[3] + o[2] * fj[6]));
                ay = 0.5 * ((fj[1] - fg[1]) + (o[0] * fj[1] + o[1] * fj[4] + o[2] * fj[7]));
                az = 0.5 * ((fj[2] - fg[2]) + (o[0] * fj[2] + o[1] * fj[5] + o[2] * fj[8]));
                w = rho[(int64_t)j * ptot + cidx];
            }
            smem4[idx] = make_double4(-2.0 * ax, -2.0 * ay, -2.0 * az, ax * ax + ay * ay + az * az);
            srho[idx] = w;
        }
        __syncthreads();
        const int nst = cl16 >> 4;
        const double* sm = reinterpret_cast<const double*>(smem4);
        for (int rt = wave; rt < nrt; rt += 4) {
            // A(i, k): component k of grid point 16 rt + i (1 for k = 3); C: |z|^2 of this lane's rows
            const int ra = rt * 16 + c;
            const double aop = kq == 3 ? 1.0 : (ra < q ? zg[3 * ra + kq] : 0.0);
            v4d_t cin;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + kq + 4 * r;
                double z2 = 0.0;
                if (row < q) {
                    const double* z = zg + 3 * row;
                    z2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                }
                cin[r] = z2;
            }
            double acc[4] = {0.0, 0.0, 0.0, 0.0}, ace[4] = {0.0, 0.0, 0.0, 0.0};
            // software pipeline: the next tile's product is in flight on the
            // matrix core while this tile's Green's functions are evaluated
            v4d_t hn = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, sm[4 * c + kq], cin, 0, 0, 0);
            double wn = srho[c];
            for (int st = 0; st < nst; ++st) {
                const v4d_t h = hn;
                const double w = wn;
                if (st + 1 < nst) {
                    hn = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, sm[4 * ((st + 1) * 16 + c) + kq], cin, 0, 0, 0);
                    wn = srho[(st + 1) * 16 + c];
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    double de;
                    const double gs = green64_grid_split<PROB>(h[r], ltab, de);
                    acc[r] = fma(gs, w, acc[r]);
                    ace[r] = fma(de, w, ace[r]);
                }
            }
            // sum over the 16 source columns (the lanes with the same kq)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = fma(-kLn2Hi, ace[r], fma(-kLn2Lo, ace[r], acc[r]));
                for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
                const int row = rt * 16 + kq + 4 * r;
                if (c == 0 && row < q) red[row] += v;
            }
        }
    }
    __syncthreads();
    const int64_t off = it_off[item];
    for (int t = threadIdx.x; t < q; t += blockDim.x) part[off + t] = red[t];
}

template <int PROB>
__global__ __launch_bounds__(256) void k_p2l32_mfma(const int* __restrict__ it_grid, const int* __restrict__ it_src0,
                                                    const int* __restrict__ it_src1, const int64_t* __restrict__ it_off,
                                                    const int* __restrict__ src, const double* __restrict__ g_frame,
                                                    const int* __restrict__ g_nr, const int* __restrict__ g_nt,
                                                    TabRuns tr, const int* __restrict__ t_off,
                                                    const int* __restrict__ t_p, const double* __restrict__ frames,
                                                    const float* __restrict__ skel_off, const float* __restrict__ rho,
                                                    int ptot, float* __restrict__ part,
                                                    const int* __restrict__ it_type, const int* __restrict__ t_col,
                                                    int ntab, const int* __restrict__ it_cfg,
                                                    const int* __restrict__ live, const int64_t* __restrict__ g_off,
                                                    const float* __restrict__ gpt, const int* __restrict__ it_list) {
    __shared__ float4 smem4[kStage];
    __shared__ float srho[kStage];
    __shared__ double red[kMaxGridQ];
    const int item = it_list ? it_list[blockIdx.x] : (int)blockIdx.x;
    if (live && !live[it_cfg[item]]) return;
    const int g = it_grid[item];
    const int q = g_nr[g] * g_nt[g];
    __shared__ StageRuns sruns;
    const int total = load_runs(sruns, tr, item, it_src1[item], it_type ? it_type[item] * ntab : 0, t_off, t_col, t_p);
    const double* fg = g_frame + 9 * (int64_t)g;
    const float* zg = gpt + 3 * g_off[g];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, c = lane & 15, kq = lane >> 4;
    const int nrt = (q + 15) >> 4;
    for (int t = threadIdx.x; t < q; t += blockDim.x) red[t] = 0.0;
    constexpr float kLn2 = 0.69314718055994530942f;
    for (int c0 = 0; c0 < total; c0 += kStage) {
        const int cl = min(kStage, total - c0);
        const int cl16 = (cl + 15) & ~15;
        __syncthreads();
        for (int idx = threadIdx.x; idx < cl16; idx += blockDim.x) {
            float ax = 8.0f, ay = 8.0f, az = 8.0f, w = 0.0f;
            if (idx < cl) {
                int sidx, oidx, cidx;
                run_point(sruns, c0 + idx, sidx, oidx, cidx);
                const int j = src[sidx];
                const double* fj = frames + 9 * (int64_t)j;
                const float* o = skel_off + 3 * (int64_t)oidx;
                ax = 0.5f * ((float)(fj[0] - fg[0]) + (o[0] * (float)fj[0] + o[1] * (float)fj[3] + o[2] * (float)fj[6]));
                ay = 0.5f * ((float)(fj[1] - fg[1]) + (o[0] * (float)fj[1] + o[1] * (float)fj[4] + o[2] * (float)fj[7]));
                az = 0.5f * ((float)(fj[2] - fg[2]) + (o[0] * (float)fj[2] + o[1] * (float)fj[5] + o[2] * (float)fj[8]));
                w = rho[(int64_t)j * ptot + cidx];
            }
            smem4[idx] = make_float4(-2.0f * ax, -2.0f * ay, -2.0f * az, ax * ax + ay * ay + az * az);
            srho[idx] = w;
        }
        __syncthreads();
        const int nst = cl16 >> 4;
        const float* sm = reinterpret_cast<const float*>(smem4);
        for (int rt = wave; rt < nrt; rt += 4) {
            const int ra = rt * 16 + c;
            const float aop = kq == 3 ? 1.0f : (ra < q ? zg[3 * ra + kq] : 0.0f);
            v4f_t cin;
            // FP32 16x16x4 layout: this lane's rows are 4 kq + r
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + 4 * kq + r;
                float z2 = 0.0f;
                if (row < q) {
                    const float* z = zg + 3 * row;
                    z2 = z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
                }
                cin[r] = z2;
            }
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            // FP32 sums over at most 64 tiles (64 terms per lane), carried in FP64
            for (int st0 = 0; st0 < nst; st0 += 64) {
                const int st1 = min(nst, st0 + 64);
                float aw[4] = {0.0f, 0.0f, 0.0f, 0.0f}, al[4] = {0.0f, 0.0f, 0.0f, 0.0f};
                v4f_t hn = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, sm[4 * (st0 * 16 + c) + kq], cin, 0, 0, 0);
                float wn = srho[st0 * 16 + c];
                for (int st = st0; st < st1; ++st) {
                    const v4f_t h = hn;
                    const float sw = wn;
                    if (st + 1 < st1) {
                        hn = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, sm[4 * ((st + 1) * 16 + c) + kq], cin, 0, 0, 0);
                        wn = srho[(st + 1) * 16 + c];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        float w, l2;
                        green32_parts_half<PROB>(h[r], w, l2);
                        aw[r] = fmaf(w, sw, aw[r]);
                        al[r] = fmaf(l2, sw, al[r]);
                    }
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] += (double)(aw[r] - kLn2 * al[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double v = acc[r];
                for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
                const int row = rt * 16 + 4 * kq + r;
                if (c == 0 && row < q) red[row] += v;
            }
        }
    }
    __syncthreads();
    const int64_t off = it_off[item];
    for (int t = threadIdx.x; t < q; t += blockDim.x) part[off + t] = (float)red[t];
}

// ------------------------------------------------------------------ L2T
// One block per patch: evaluate every grid of the patch's list at the patch's
// K* nodes, in the grid's stereographic polar coordinates (tan(phi/2) / Tc,
// theta), and add the total into U once. The expansion of a grid is
//     sum_k [cos k theta C_k(x) + sin k theta S_k(x)],
// C_k, S_k Chebyshev series over the degrees of the parity of k. Per grid, a
// thread forms the Chebyshev values of its nodes once per parity and reuses
// them for every angular row of that parity; cos k theta and sin k theta of
// one parity follow the three-term recurrence f_{k+2} = 2 cos 2theta f_k -
// f_{k-2} (one fma each, the two newest values leapfrogging so that no
// register moves are needed). Coefficients are staged in LDS through a double
// buffer filled from registers loaded one grid ahead, so the next grid's
// global loads are in flight while the current one is summed and each grid
// costs one barrier.
// LDS per buffer: a grid's coefficients; at the end (fused P apply) the
// node values and angular coefficients of the largest basis (M = 15: 16 x 36
// + 31 x 16 values)
constexpr int kL2tBuf = kMaxGridQ;
static_assert(16 * 36 + 31 * 16 <= 2 * kL2tBuf, "fused P apply does not fit the L2T buffers");

template <class T, int NPT, int NR>
__device__ __forceinline__ void l2t_row(const T* __restrict__ cs, int half, int k, const T (&tb)[NPT][NR],
                                        const T (&ck)[NPT], const T (&sk)[NPT], T (&val)[NPT]) {
    const T* cc = cs + k * NR;
    T rc[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) rc[r] = cc[0] * tb[r][0];
#pragma unroll
    for (int n = 1; n < NR; ++n) {
        const T cv = cc[n];
#pragma unroll
        for (int r = 0; r < NPT; ++r) rc[r] += cv * tb[r][n];
    }
    if (k > 0 && k < half) {
        const T* sc = cs + (half + k) * NR;
        T rs[NPT];
#pragma unroll
        for (int r = 0; r < NPT; ++r) rs[r] = sc[0] * tb[r][0];
#pragma unroll
        for (int n = 1; n < NR; ++n) {
            const T sv = sc[n];
#pragma unroll
            for (int r = 0; r < NPT; ++r) rs[r] += sv * tb[r][n];
        }
#pragma unroll
        for (int r = 0; r < NPT; ++r) val[r] += ck[r] * rc[r] + sk[r] * rs[r];
    } else {
#pragma unroll
        for (int r = 0; r < NPT; ++r) val[r] += ck[r] * rc[r];
    }
}

template <class T, int NPT, int NR>
__device__ __forceinline__ void l2t_sum(const T* __restrict__ cs, int half, const T (&xs)[NPT],
                                        const T (&ct)[NPT], const T (&st)[NPT], T (&val)[NPT]) {
    T c2[NPT], s2[NPT], t2[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        c2[r] = ct[r] * ct[r] - st[r] * st[r];
        s2[r] = T(2) * ct[r] * st[r];
        t2[r] = T(2) * c2[r];
    }
#pragma unroll
    for (int par = 0; par < 2; ++par) {
        // tb[r][n] = T_{2n+par}(x): T_{m+2} = 2 T_2 T_m - T_{m-2}, T_2 = 2 x^2 - 1
        T tb[NPT][NR], ca[NPT], sa[NPT], cb[NPT], sb[NPT];
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const T x = xs[r], y = T(2) * x * x - T(1), ty = T(2) * y;
            tb[r][0] = par ? x : T(1);
            if (NR > 1) tb[r][1] = par ? x * (ty - T(1)) : y;
#pragma unroll
            for (int n = 2; n < NR; ++n) tb[r][n] = ty * tb[r][n - 1] - tb[r][n - 2];
            // (ca, sa) = cos, sin of k theta; (cb, sb) = of (k - 2) theta
            ca[r] = par ? ct[r] : T(1);
            sa[r] = par ? st[r] : T(0);
            cb[r] = par ? ct[r] : c2[r];
            sb[r] = par ? -st[r] : -s2[r];
        }
        for (int k = par; k <= half; k += 4) {
            l2t_row<T, NPT, NR>(cs, half, k, tb, ca, sa, val);
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                cb[r] = t2[r] * ca[r] - cb[r];
                sb[r] = t2[r] * sa[r] - sb[r];
            }
            if (k + 2 > half) break;
            l2t_row<T, NPT, NR>(cs, half, k + 2, tb, cb, sb, val);
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                ca[r] = t2[r] * cb[r] - ca[r];
                sa[r] = t2[r] * sb[r] - sa[r];
            }
        }
    }
}

template <class T>
__device__ __forceinline__ T rsqrt_t(T v) {
    if constexpr (sizeof(T) == 8) return rsqrt64(v);
    else return rsqrtf(v);
}


template <class T, int NPT>
__global__ __launch_bounds__(512 / NPT) void k_l2t(int Kstar, const double* __restrict__ frames,
                                                    const T* __restrict__ node_off, const int64_t* __restrict__ l2t_ptr,
                                                    const int* __restrict__ l2t_grid, const double* __restrict__ g_frame,
                                                    const double* __restrict__ g_T, const int* __restrict__ g_nr,
                                                    const int* __restrict__ g_nt, const int64_t* __restrict__ g_off,
                                                    const T* __restrict__ coef, T* __restrict__ U,
                                                    const int* __restrict__ pt_cfg, const int* __restrict__ live,
                                                    const int* __restrict__ ptype, int node_stride, PApply<T> pa,
                                                    const int* __restrict__ g_same) {
    constexpr int kThreads = 512 / NPT;
    constexpr int kPre = (kMaxGridQ + kThreads - 1) / kThreads;  // coefficients per thread per grid
    // the grid coefficients' double buffer; at the end (fused P apply) the
    // node values, the trig rows and the angular coefficients
    __shared__ __align__(16) T cs_all[2 * kL2tBuf];
    const int i = blockIdx.x;
    if (live && !live[pt_cfg[i]]) return;
    const int64_t a0 = l2t_ptr[i], a1 = l2t_ptr[i + 1];
    if (a0 == a1 && !pa.y) return;
    if (ptype) node_off += (int64_t)ptype[i] * node_stride;
    const double* fi = frames + 9 * (int64_t)i;
    T ox[NPT], oy[NPT], oz[NPT], val[NPT];
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int q = threadIdx.x + r * kThreads;
        ox[r] = oy[r] = oz[r] = val[r] = T(0);
        if (q < Kstar) {
            const T o0 = node_off[3 * q], o1 = node_off[3 * q + 1], o2 = node_off[3 * q + 2];
            ox[r] = o0 * (T)fi[0] + o1 * (T)fi[3] + o2 * (T)fi[6];
            oy[r] = o0 * (T)fi[1] + o1 * (T)fi[4] + o2 * (T)fi[7];
            oz[r] = o0 * (T)fi[2] + o1 * (T)fi[5] + o2 * (T)fi[8];
        }
    }
    // coefficients of the next grid, loaded into registers ahead of use
    T pre[kPre];
    auto fetch = [&](int g) {
        const int q = g_nr[g] * g_nt[g];
        const T* src = coef + g_off[g];
#pragma unroll
        for (int j = 0; j < kPre; ++j) {
            const int t = threadIdx.x + j * kThreads;
            pre[j] = t < q ? src[t] : T(0);
        }
    };
    int gn = a0 < a1 ? l2t_grid[a0] : 0;
    if (a0 < a1) fetch(gn);
    int buf = 0;
    // stereographic polar coordinates of the nodes about the current cap; a
    // grid over the same cap as the one before keeps them
    T xs[NPT], ct[NPT], st[NPT];
    int gprev = -2;
    for (int64_t aa = a0; aa < a1; ++aa) {
        const int g = gn;
#pragma unroll
        for (int j = 0; j < kPre; ++j) cs_all[buf * kL2tBuf + threadIdx.x + j * kThreads] = pre[j];
        __syncthreads();
        if (aa + 1 < a1) {
            gn = l2t_grid[aa + 1];
            fetch(gn);
        }
        const int nr = g_nr[g], half = g_nt[g] / 2;
        const bool same_cap = g == gprev + 1 && g_same[g];
        gprev = g;
        if (!same_cap) {
            const double* fg = g_frame + 9 * (int64_t)g;
            const T dcx = (T)(fi[0] - fg[0]), dcy = (T)(fi[1] - fg[1]), dcz = (T)(fi[2] - fg[2]);
            const T e1x = (T)fg[3], e1y = (T)fg[4], e1z = (T)fg[5];
            const T e2x = (T)fg[6], e2y = (T)fg[7], e2z = (T)fg[8];
            const T invT = (T)(1.0 / g_T[g]);
            // stereographic polar coordinates of every node about the grid's cap
            // centre: for v = node - centre (both on the unit sphere) at angle
            // phi, |v|^2 = 2 - 2 cos phi and the in-plane part has length sin phi,
            // so tan(phi / 2) = (1 - cos phi) / sin phi = |v|^2 / (2 sin phi):
            // one reciprocal square root per node and grid, no cancellation
#pragma unroll
            for (int r = 0; r < NPT; ++r) {
                const T vx = dcx + ox[r], vy = dcy + oy[r], vz = dcz + oz[r];
                const T x1 = vx * e1x + vy * e1y + vz * e1z;
                const T x2 = vx * e2x + vy * e2y + vz * e2z;
                const T s = x1 * x1 + x2 * x2;
                const bool off_axis = s > T(0);
                const T w = rsqrt_t<T>(off_axis ? s : T(1));
                ct[r] = off_axis ? x1 * w : T(1);
                st[r] = off_axis ? x2 * w : T(0);
                const T v2 = vx * vx + vy * vy + vz * vz;
                const T x = off_axis ? T(0.5) * v2 * w * invT : T(0);
                xs[r] = x > T(1) ? T(1) : x;
            }
        }
        const T* c = cs_all + buf * kL2tBuf;
        static_assert(kMaxGridNr == 16, "one case per radial order");
        switch (nr) {
#define NCE_L2T_CASE(n) \
    case n: l2t_sum<T, NPT, n>(c, half, xs, ct, st, val); break;
            NCE_L2T_CASE(1) NCE_L2T_CASE(2) NCE_L2T_CASE(3) NCE_L2T_CASE(4)
            NCE_L2T_CASE(5) NCE_L2T_CASE(6) NCE_L2T_CASE(7) NCE_L2T_CASE(8)
#undef NCE_L2T_CASE
            // long radial series (grids tighter than about 1e-9): one node at a
            // time, so the Chebyshev values of all NPT nodes need not be live
#define NCE_L2T_CASE(n)                                                       \
    case n:                                                                   \
        for (int r = 0; r < NPT; ++r) {                                       \
            T x1[1] = {xs[r]}, c1[1] = {ct[r]}, s1[1] = {st[r]}, v1[1] = {val[r]}; \
            l2t_sum<T, 1, n>(c, half, x1, c1, s1, v1);                        \
            val[r] = v1[0];                                                   \
        }                                                                     \
        break;
            NCE_L2T_CASE(9) NCE_L2T_CASE(10) NCE_L2T_CASE(11) NCE_L2T_CASE(12)
            NCE_L2T_CASE(13) NCE_L2T_CASE(14) NCE_L2T_CASE(15) NCE_L2T_CASE(16)
#undef NCE_L2T_CASE
            default: break;
        }
        buf ^= 1;
    }
    if (!pa.y) {
#pragma unroll
        for (int r = 0; r < NPT; ++r) {
            const int qn = threadIdx.x + r * kThreads;
            if (qn < Kstar) U[(int64_t)i * Kstar + qn] += val[r];
        }
        return;
    }
    // Step 5 in the epilogue: u = U (the near field) + the interpolated far
    // field stays in LDS, and y_i = x_i + P u through P's two factors: an
    // angular transform per ring of nodes, F[j][a] = sum_b trig[j][b] u[a][b],
    // then a radial sum per basis function, (P u)_k = sum_a rad[k][a] F[mode_k][a]
    const int M = pa.M, nrad = M + 1, nth = 2 * M + 2, nmode = 2 * M + 1;
    constexpr int W = 16 / sizeof(T);           // values per 16-byte read
    constexpr int kMaxV = 32 / W;               // 16-byte reads per ring (nth <= 32)
    const int nv = (nth + W - 1) / W, ld = nv * W + 4;
    T* su = cs_all;                             // 16 x ld node values, zero padded to nv W
    T* sf = su + 16 * ld;                       // nmode x 16 angular coefficients
    __syncthreads();                            // the last grid's coefficients are consumed
    const float inv_nth = __builtin_amdgcn_rcpf((float)nth);
#pragma unroll
    for (int r = 0; r < NPT; ++r) {
        const int qn = threadIdx.x + r * kThreads;
        if (qn < Kstar) {
            const int a = div_small(qn, inv_nth), b = qn - a * nth;
            su[a * ld + b] = U[(int64_t)i * Kstar + qn] + val[r];
        }
    }
    if (nv * W > nth)
        for (int t = threadIdx.x; t < nrad * W; t += kThreads) {
            const int a = t / W, e = nth + t % W;
            if (e < nv * W) su[a * ld + e] = T(0);
        }
    __syncthreads();
    typedef T vec_t __attribute__((ext_vector_type(W)));
    {
        // thread (ring a, modes j = j0, j0 + kThreads / 16, ...): the ring's
        // values stay in registers; the trig rows (zero padded to trig_ld)
        // come from the cache
        const int a = threadIdx.x & 15;
        if (a < nrad) {
            vec_t u[kMaxV];
            const vec_t* ur = reinterpret_cast<const vec_t*>(su + a * ld);
#pragma unroll
            for (int v = 0; v < kMaxV; ++v)
                if (v < nv) u[v] = ur[v];
            for (int j = threadIdx.x >> 4; j < nmode; j += kThreads >> 4) {
                const vec_t* tr = reinterpret_cast<const vec_t*>(pa.trig + (int64_t)j * pa.trig_ld);
                T acc = T(0);
#pragma unroll
                for (int v = 0; v < kMaxV; ++v)
                    if (v < nv) {
                        const vec_t c = tr[v];
#pragma unroll
                        for (int e = 0; e < W; ++e) acc += c[e] * u[v][e];
                    }
                sf[j * 16 + a] = acc;
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < pa.K; k += kThreads) {
        const T* rr = pa.rad + (int64_t)k * nrad;
        const T* fr = sf + pa.mode[k] * 16;
        T acc = T(0);
        for (int a = 0; a < nrad; ++a) acc += rr[a] * fr[a];
        const int64_t e = (int64_t)i * pa.K + k;
        pa.y[e] = pa.x[e] + (double)acc;
    }
}

template <class T>
T* dev_copy(const std::vector<T>& v) {
    T* p = nullptr;
    if (v.empty()) return nullptr;
    if (hipMalloc((void**)&p, v.size() * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    if (hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
        throw std::runtime_error("hipMemcpy failed (tree upload)");
    return p;
}

template <class T>
T* dev_alloc(int64_t n) {
    T* p = nullptr;
    if (n <= 0) return nullptr;
    if (hipMalloc((void**)&p, (size_t)n * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    return p;
}

}  // namespace

void upload_tree(const Tree& t, int Kstar, int p, const std::vector<int>& tab_off, const std::vector<int>& tab_p,
                 hipStream_t s, DeviceTree& d, const TypeLayout* tl) {
    d.ngrid = t.ngrid;
    d.max_q = t.max_q;
    d.g_table = dev_copy(t.g_table);
    if (tl) {
        // strength row length: the longest type's tables
        int ldr = 0;
        const int ntype = (int)tl->t_p.size() / tl->ntab;
        for (int ty = 0; ty < ntype; ++ty) {
            const int b = ty * tl->ntab + tl->ntab - 1;
            ldr = std::max(ldr, tl->t_col[b] + tl->t_p[b]);
        }
        d.ptot = ldr;
        d.t_off = dev_copy(tl->t_soff);
        d.t_col = dev_copy(tl->t_col);
        d.t_p = dev_copy(tl->t_p);
        d.ptype = dev_copy(tl->ptype);
        d.it_type = dev_copy(t.it_type);
        d.ntab = tl->ntab;
        d.node_stride = tl->node_stride;
    } else {
        d.ptot = tab_off.back() + tab_p.back();
        d.t_off = dev_copy(tab_off);
        d.t_p = dev_copy(tab_p);
    }
    d.nitems = (int)t.it_grid.size();
    d.N = t.N;
    d.Kstar = Kstar;
    d.p = p;
    d.g_frame = dev_copy(t.g_frame);
    {
        std::vector<double> tc(t.g_R.size());
        for (size_t g = 0; g < tc.size(); ++g) tc[g] = std::tan(0.5 * t.g_R[g]);
        d.g_T = dev_copy(tc);
    }
    d.g_nr = dev_copy(t.g_nr);
    d.g_nt = dev_copy(t.g_nt);
    d.g_off = dev_copy(t.g_off);
    d.g_item0 = dev_copy(t.g_item0);
    d.g_item1 = dev_copy(t.g_item1);
    d.it_grid = dev_copy(t.it_grid);
    d.it_src0 = dev_copy(t.it_src0);
    d.it_src1 = dev_copy(t.it_src1);
    d.it_off = dev_copy(t.it_off);
    d.p2l_src = dev_copy(t.p2l_src);
    d.dl_ptr = dev_copy(t.dl_ptr);
    d.dl_src = dev_copy(t.dl_src);
    d.l2t_ptr = dev_copy(t.l2t_ptr);
    d.l2t_grid = dev_copy(t.l2t_grid);
    d.it_cfg = dev_copy(t.it_cfg);
    d.g_cfg = dev_copy(t.g_cfg);
    d.pt_cfg = dev_copy(t.pt_cfg);
    {
        // items that are their grid's only one finish the grid themselves
        std::vector<int> solo(t.it_grid.size(), 0), multi;
        for (int g = 0; g < t.ngrid; ++g) {
            if (t.g_item1[g] - t.g_item0[g] == 1) solo[t.g_item0[g]] = 1;
            else if (t.g_item1[g] > t.g_item0[g]) multi.push_back(g);
        }
        d.it_solo = dev_copy(solo);
        d.n_multi = (int)multi.size();
        d.g_multi = dev_copy(multi);
        // transform tables per distinct (nr, nt): cos, sin(2 pi j / nt), cos(2 pi j / (8 nr))
        std::map<std::pair<int, int>, int> at;
        std::vector<double> tt;
        std::vector<int> gt(t.ngrid);
        for (int g = 0; g < t.ngrid; ++g) {
            const int nr = t.g_nr[g], nt = t.g_nt[g];
            auto it = at.find({nr, nt});
            if (it == at.end()) {
                it = at.emplace(std::make_pair(nr, nt), (int)tt.size()).first;
                for (int j = 0; j < nt; ++j) tt.push_back(std::cos(2.0 * kPi * j / nt));
                for (int j = 0; j < nt; ++j) tt.push_back(std::sin(2.0 * kPi * j / nt));
                for (int j = 0; j < 8 * nr; ++j) tt.push_back(std::cos(2.0 * kPi * j / (8.0 * nr)));
            }
            gt[g] = it->second;
        }
        d.ttab = dev_copy(tt);
        d.g_ttab = dev_copy(gt);
    }
    d.coef64 = dev_alloc<double>(t.total_q);
    d.part64 = dev_alloc<double>(t.total_partial);
    d.coef32 = dev_alloc<float>(t.total_q);
    d.part32 = dev_alloc<float>(t.total_partial);
    {
        // busy (target, source split) slots of a block, as p2l_layout arranges them:
        // ns = 256 / ceil(q / R) splits of q targets over 256 R slots
        std::vector<int> l4, l8;
        for (int it = 0; it < (int)t.it_grid.size(); ++it) {
            const int q = t.g_nr[t.it_grid[it]] * t.g_nt[t.it_grid[it]];
            auto use = [&](int R) {
                const int qq = (q + R - 1) / R;
                const int ns = std::min(64, std::max(1, 256 / std::max(qq, 1)));
                return (double)std::min(ns * q, 256 * R) / (256.0 * R);
            };
            if (q <= 1024 && use(4) >= use(8)) l4.push_back(it);
            else l8.push_back(it);
        }
        d.n_items4 = (int)l4.size();
        d.items4 = dev_copy(l4);
        d.items8 = dev_copy(l8);
    }
    {
        std::vector<LogEntry> lt(kLogTab);
        build_log_table(lt.data());
        d.logtab = dev_copy(lt);
        // the octaves of every item's logarithm window
        static_assert(kWinOct == kLogWindowOctaves, "the tree's windows are the kernels'");
        if (t.it_win.size() != t.it_grid.size()) throw std::runtime_error("P2L items without logarithm windows");
        int lo = 0, hi = 0;
        for (size_t it = 0; it < t.it_win.size(); ++it) {
            lo = it ? std::min(lo, t.it_win[it]) : t.it_win[it];
            hi = it ? std::max(hi, t.it_win[it]) : t.it_win[it];
        }
        std::vector<LogEntry> wt((size_t)(hi - lo + kWinOct) * kWinBins);
        build_log_window_table(lo, hi - lo + kWinOct, wt.data());
        d.win_first = lo;
        d.logwin = dev_copy(wt);
        d.it_win = dev_copy(t.it_win);
    }
    {
        // grids over the same cap as the grid before them (a box's near- and
        // far-source grids): the interpolation keeps the nodes' polar coordinates
        std::vector<int> same(t.ngrid, 0);
        for (int g = 1; g < t.ngrid; ++g)
            same[g] = t.g_R[g] == t.g_R[g - 1] &&
                      std::equal(t.g_frame.begin() + 9 * (size_t)g, t.g_frame.begin() + 9 * (size_t)g + 9,
                                 t.g_frame.begin() + 9 * (size_t)(g - 1));
        d.g_same = dev_copy(same);
    }
    {
        // runs of one outgoing table in every item's sources
        if (t.p2l_tab.size() != t.p2l_src.size()) throw std::runtime_error("P2L sources without outgoing tables");
        std::vector<int> r0(t.it_grid.size() + 1, 0), rs, rt;
        for (size_t it = 0; it < t.it_grid.size(); ++it) {
            r0[it] = (int)rs.size();
            for (int q = t.it_src0[it]; q < t.it_src1[it]; ++q)
                if (q == t.it_src0[it] || t.p2l_tab[q] != t.p2l_tab[q - 1]) {
                    rs.push_back(q);
                    rt.push_back(t.p2l_tab[q]);
                }
            if ((int)rs.size() - r0[it] > kMaxTableRuns) throw std::runtime_error("P2L item with too many table runs");
        }
        r0.back() = (int)rs.size();
        d.it_run0 = dev_copy(r0);
        d.run_src = dev_copy(rs);
        d.run_tab = dev_copy(rt);
    }
    d.gpt64 = dev_alloc<double>(3 * t.total_q);
    d.gpt32 = dev_alloc<float>(3 * t.total_q);
    if (d.ngrid > 0) {
        hipLaunchKernelGGL(k_grid_points, dim3(d.ngrid), dim3(256), 0, s, d.g_nr, d.g_nt, d.g_T, d.g_frame, d.g_off,
                           d.gpt64, d.gpt32);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            throw std::runtime_error("grid point setup failed");
    }
}

void free_tree(DeviceTree& d) {
    void* ptrs[] = {d.g_table, d.t_off, d.t_p, d.g_frame, d.g_T,   d.g_nr,     d.g_nt,     d.g_off,  d.g_item0, d.g_item1,
                    d.it_grid, d.it_src0, d.it_src1, d.it_off,  d.p2l_src, d.dl_ptr, d.dl_src,
                    d.l2t_ptr, d.l2t_grid, d.it_solo, d.coef64,  d.part64, d.g_multi,  d.coef32, d.part32, d.ttab, d.g_ttab,
                    d.it_cfg, d.g_cfg, d.pt_cfg, d.gpt64, d.gpt32, d.items4, d.items8, d.logtab,
                    d.it_type, d.t_col, d.ptype, d.it_win, d.logwin, d.it_run0, d.run_src, d.run_tab, d.g_same};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    d = DeviceTree();
}

template <class T, int PROB, int R>
void launch_p2l(hipStream_t s, const DeviceTree& d, const double* frames, const T* skel_off, const T* rho,
                const int* live, int nblocks, const int* it_list) {
    if (nblocks <= 0) return;
    if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL((k_p2l64<PROB, R>), dim3(nblocks), dim3(256), 0, s, d.it_grid, d.it_src0, d.it_src1,
                           d.it_off, d.p2l_src, d.g_frame, d.g_T, d.g_nr, d.g_nt, TabRuns{d.it_run0, d.run_src, d.run_tab}, d.t_off, d.t_p, frames,
                           skel_off, rho, d.ptot, d.part64, d.it_type, d.t_col, d.ntab, d.it_cfg, live, d.g_off, d.gpt64,
                           it_list, d.it_win, d.logwin, d.win_first, d.it_solo, d.coef64, d.ttab, d.g_ttab);
    else
        hipLaunchKernelGGL((k_p2l32<PROB, R>), dim3(nblocks), dim3(256), 0, s, d.it_grid, d.it_src0, d.it_src1,
                           d.it_off, d.p2l_src, d.g_frame, d.g_T, d.g_nr, d.g_nt, TabRuns{d.it_run0, d.run_src, d.run_tab}, d.t_off, d.t_p, frames,
                           skel_off, rho, d.ptot, d.part32, d.it_type, d.t_col, d.ntab, d.it_cfg, live, d.g_off, d.gpt32,
                           it_list, d.it_solo, d.coef32, d.ttab, d.g_ttab);
}

template <class T, int PROB>
void launch_p2l_mfma(hipStream_t s, const DeviceTree& d, const double* frames, const T* skel_off, const T* rho,
                     const int* live) {
    if constexpr (sizeof(T) == 8)
        hipLaunchKernelGGL((k_p2l64_mfma<PROB>), dim3(d.nitems), dim3(256), 0, s, d.it_grid, d.it_src0, d.it_src1,
                           d.it_off, d.p2l_src, d.g_frame, d.g_nr, d.g_nt, TabRuns{d.it_run0, d.run_src, d.run_tab}, d.t_off, d.t_p, frames, skel_off,
                           rho, d.ptot, d.part64, d.it_type, d.t_col, d.ntab, d.it_cfg, live, d.g_off, d.gpt64,
                           (const int*)nullptr, d.logtab);
    else
        hipLaunchKernelGGL((k_p2l32_mfma<PROB>), dim3(d.nitems), dim3(256), 0, s, d.it_grid, d.it_src0, d.it_src1,
                           d.it_off, d.p2l_src, d.g_frame, d.g_nr, d.g_nt, TabRuns{d.it_run0, d.run_src, d.run_tab}, d.t_off, d.t_p, frames, skel_off,
                           rho, d.ptot, d.part32, d.it_type, d.t_col, d.ntab, d.it_cfg, live, d.g_off, d.gpt32,
                           (const int*)nullptr);
}

template <class T, int PROB>
void launch_p2l_shape(hipStream_t s, const DeviceTree& d, const double* frames, const T* skel_off, const T* rho,
                      const int* live, int r_tgt) {
    if (r_tgt == 16) {
        launch_p2l_mfma<T, PROB>(s, d, frames, skel_off, rho, live);
    } else if (r_tgt == 8) {
        launch_p2l<T, PROB, 8>(s, d, frames, skel_off, rho, live, d.nitems, nullptr);
    } else if (r_tgt == 4) {
        launch_p2l<T, PROB, 4>(s, d, frames, skel_off, rho, live, d.nitems, nullptr);
    } else {
        // per item: the shape that keeps more (target, source split) slots busy
        launch_p2l<T, PROB, 4>(s, d, frames, skel_off, rho, live, d.n_items4, d.items4);
        launch_p2l<T, PROB, 8>(s, d, frames, skel_off, rho, live, d.nitems - d.n_items4, d.items8);
    }
}

template <class T>
hipError_t tree_far(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* skel_off,
                    const T* rho, const int* live, int r_tgt) {
    if (!d.it_cfg) live = nullptr;
    if (r_tgt != 4 && r_tgt != 8 && r_tgt != 0 && r_tgt != 16) return hipErrorInvalidValue;
    if (r_tgt != 16 && d.max_q > 256 * (r_tgt == 4 ? 4 : 8)) return hipErrorInvalidValue;
    if (d.nitems > 0) {
        if (problem == 1) launch_p2l_shape<T, 1>(s, d, frames, skel_off, rho, live, r_tgt);
        else launch_p2l_shape<T, 0>(s, d, frames, skel_off, rho, live, r_tgt);
    }
    // the vector-unit shapes finish the grids of one item in the P2L block;
    // the others (every grid after the matrix-core shape) are reduced here
    const int* glist = r_tgt == 16 ? nullptr : d.g_multi;
    const int nred = r_tgt == 16 ? d.ngrid : d.n_multi;
    if (nred > 0) {
        if constexpr (sizeof(T) == 8)
            hipLaunchKernelGGL((k_reduce_coef<double>), dim3(nred), dim3(256), 0, s, glist, d.g_nr, d.g_nt, d.g_off,
                               d.g_item0, d.g_item1, d.it_off, d.part64, d.coef64, d.g_cfg, live, d.ttab, d.g_ttab);
        else
            hipLaunchKernelGGL((k_reduce_coef<float>), dim3(nred), dim3(256), 0, s, glist, d.g_nr, d.g_nt, d.g_off,
                               d.g_item0, d.g_item1, d.it_off, d.part32, d.coef32, d.g_cfg, live, d.ttab, d.g_ttab);
    }
    return hipGetLastError();
}
template hipError_t tree_far<double>(hipStream_t, const DeviceTree&, int, const double*, const double*,
                                     const double*, const int*, int);
template hipError_t tree_far<float>(hipStream_t, const DeviceTree&, int, const double*, const float*, const float*,
                                    const int*, int);

template <class T>
hipError_t tree_near(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* node_off,
                     const T* skel_off, const T* rho, T* U, const int* live) {
    if (!d.pt_cfg) live = nullptr;
    // near field uses the base table (the first p columns of every strength row)
    TypeTabs tt;
    if (d.ptype) {
        tt.ptype = d.ptype;
        tt.t_soff = d.t_off;
        tt.t_col = d.t_col;
        tt.t_p = d.t_p;
        tt.ntab = d.ntab;
        tt.node_stride = d.node_stride;
    }
    return list_sum<T>(s, problem, (int)d.N, d.Kstar, d.p, frames, node_off, skel_off, rho, d.ptot, U, d.dl_ptr,
                       d.dl_src, d.logtab, d.pt_cfg, live, tt);
}
template hipError_t tree_near<double>(hipStream_t, const DeviceTree&, int, const double*, const double*,
                                      const double*, const double*, double*, const int*);
template hipError_t tree_near<float>(hipStream_t, const DeviceTree&, int, const double*, const float*, const float*,
                                     const float*, float*, const int*);

template <class T>
hipError_t tree_interp(hipStream_t s, const DeviceTree& d, const double* frames, const T* node_off, T* U,
                       const int* live, int npt, const PApply<T>* pa) {
    PApply<T> p;
    if (pa) {
        p = *pa;
        if (!p.y || !p.x || !p.trig || !p.rad || !p.mode || p.M < 0 || p.M > 15 || p.trig_ld % 4 != 0 ||
            p.trig_ld < 2 * p.M + 2)
            return hipErrorInvalidValue;
    }
    if (d.ngrid == 0 && !p.y) return hipSuccess;
    if (!d.pt_cfg) live = nullptr;
    const T* coef;
    if constexpr (sizeof(T) == 8) coef = d.coef64;
    else coef = d.coef32;
    // nodes per thread x threads per block covers K*
    const int threads = npt == 2 ? 256 : (npt == 4 ? 128 : 64);
    if ((npt != 2 && npt != 4 && npt != 8) || threads * npt < d.Kstar) return hipErrorInvalidValue;
    if (npt == 2)
        hipLaunchKernelGGL((k_l2t<T, 2>), dim3((unsigned)d.N), dim3(threads), 0, s, d.Kstar, frames, node_off,
                           d.l2t_ptr, d.l2t_grid, d.g_frame, d.g_T, d.g_nr, d.g_nt, d.g_off, coef, U, d.pt_cfg, live,
                           d.ptype, d.node_stride, p, d.g_same);
    else if (npt == 4)
        hipLaunchKernelGGL((k_l2t<T, 4>), dim3((unsigned)d.N), dim3(threads), 0, s, d.Kstar, frames, node_off,
                           d.l2t_ptr, d.l2t_grid, d.g_frame, d.g_T, d.g_nr, d.g_nt, d.g_off, coef, U, d.pt_cfg, live,
                           d.ptype, d.node_stride, p, d.g_same);
    else
        hipLaunchKernelGGL((k_l2t<T, 8>), dim3((unsigned)d.N), dim3(threads), 0, s, d.Kstar, frames, node_off,
                           d.l2t_ptr, d.l2t_grid, d.g_frame, d.g_T, d.g_nr, d.g_nt, d.g_off, coef, U, d.pt_cfg, live,
                           d.ptype, d.node_stride, p, d.g_same);
    return hipGetLastError();
}
template hipError_t tree_interp<double>(hipStream_t, const DeviceTree&, const double*, const double*, double*,
                                        const int*, int, const PApply<double>*);
template hipError_t tree_interp<float>(hipStream_t, const DeviceTree&, const double*, const float*, float*,
                                       const int*, int, const PApply<float>*);

}  // namespace nce
