// Per-eps precompute on the GPU: the randomized interpolative decomposition
// of a patch's outgoing field (Section 7.1) and the modal one-patch solves
// batched over the azimuthal orders (Section 9.2).
//
// Interpolative decomposition, for training points x^t on the sphere at
// arclength >= D from the patch centre and the fine grid x^f of the patch:
//   A = G(x^t, x^f)                       (nt x nf, Green's function kernel)
//   Y = Omega A                           (ell x nf, Omega standard normal;
//                                          MFMA GEMM, A never leaves HBM)
//   Y Pi = Q R                            (Householder QR with column pivoting,
//                                          one step per launch pair, all ell
//                                          steps on the device; the rank p is
//                                          the first step whose pivot norm is
//                                          <= tol_id times the first)
//   T = Pi W B: rows of W B at the skeleton plus R11^-1 R12 times the rest.
// Modal solves: the M + 1 collocation systems A_m sigma = F_m (260 x 260, one
// LU with partial pivoting per block, all orders in one launch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "precompute.hpp"
#include "precompute_gpu.hpp"

namespace nce {
namespace {

void chk(hipError_t e, const char* what) {
    if (e != hipSuccess) throw std::runtime_error(std::string("precompute on the GPU: ") + what + ": " +
                                                  hipGetErrorString(e));
}

template <class T>
struct Buf {
    T* p = nullptr;
    size_t n = 0;
    explicit Buf(size_t count) : n(count) {
        if (count && hipMalloc((void**)&p, count * sizeof(T)) != hipSuccess) throw std::bad_alloc();
    }
    Buf(const Buf&) = delete;
    Buf& operator=(const Buf&) = delete;
    ~Buf() {
        if (p) (void)hipFree(p);
    }
    void put(const std::vector<T>& v, hipStream_t s) {
        chk(hipMemcpyAsync(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, s), "upload");
    }
    void get(std::vector<T>& v, hipStream_t s, size_t count) const {
        v.resize(count);
        chk(hipMemcpyAsync(v.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost, s), "download");
    }
};

// Standard normal numbers from a counter: splitmix64 of (seed, index) gives
// two uniforms, Box-Muller the normal.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
    z += 0x9e3779b97f4a7c15ULL;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

__global__ void k_gauss(int64_t n, uint64_t seed, double* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = splitmix64(seed ^ (2 * (uint64_t)i)), b = splitmix64(seed ^ (2 * (uint64_t)i + 1));
        const double u1 = ((double)(a >> 11) + 0.5) * 0x1.0p-53, u2 = (double)(b >> 11) * 0x1.0p-53;
        out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
}

// G on the sphere between point sets (rows x cols, row-major out[r * ldo + c]),
// the chord from coordinate differences: exterior 2/d - log(2/d) - log(1 + d/2),
// interior 2/d + log(2/d) - log(1 + d/2) (eqs. Gextonsurface, Gintonsurface).
__global__ void k_green_matrix(int problem, int rows, int cols, const double* __restrict__ xr,
                               const double* __restrict__ xc, double* __restrict__ out, int64_t ldo) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (c >= cols) return;
    const double dx = xr[3 * r] - xc[3 * c], dy = xr[3 * r + 1] - xc[3 * c + 1], dz = xr[3 * r + 2] - xc[3 * c + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double w = 2.0 / d;
    out[(int64_t)r * ldo + c] = problem == 1 ? (w - log(w) - log1p(0.5 * d)) : (w + log(w) - log1p(0.5 * d));
}

__global__ __launch_bounds__(256) void k_colnorms(int nf, int ell, const double* __restrict__ Y,
                                                  double* __restrict__ nrm, double* __restrict__ nrm0) {
    const int f = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (f >= nf) return;
    double s = 0.0;
    for (int a = lane; a < ell; a += 64) {
        const double v = Y[(int64_t)f * ell + a];
        s += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (lane == 0) nrm[f] = nrm0[f] = s;
}

// State of the pivoted QR shared by its launches: st[0] = tau of the current
// step, st[1] = |R_00|, ist[0] = stop flag, ist[1] = rank p so far.
// Step k, part 1 (one block): pick the column of largest remaining norm among
// k..nf-1 (the first on ties), swap it into place, form the Householder
// reflector of its trailing part in place (v_k = 1 implied, tau).
__global__ __launch_bounds__(1024) void k_qr_pivot(int k, int nf, int ell, double tol, double* __restrict__ Y,
                                                   double* __restrict__ nrm, double* __restrict__ nrm0,
                                                   int* __restrict__ piv, double* __restrict__ st,
                                                   int* __restrict__ ist, double* __restrict__ alphas) {
    __shared__ double bv[16];
    __shared__ int bi[16];
    __shared__ double red[16];
    if (ist[0]) return;
    double best = -1.0;
    int bj = nf;
    for (int j = k + threadIdx.x; j < nf; j += blockDim.x)
        if (nrm[j] > best) {
            best = nrm[j];
            bj = j;
        }
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_down(best, o, 64);
        const int oj = __shfl_down(bj, o, 64);
        if (ob > best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
    }
    if (threadIdx.x % 64 == 0) {
        bv[threadIdx.x / 64] = best;
        bi[threadIdx.x / 64] = bj;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)blockDim.x / 64; ++w)
            if (bv[w] > bv[0] || (bv[w] == bv[0] && bi[w] < bi[0])) {
                bv[0] = bv[w];
                bi[0] = bi[w];
            }
    }
    __syncthreads();
    const int jb = bi[0];
    double* ck = Y + (int64_t)k * ell;
    if (jb != k) {
        double* cb = Y + (int64_t)jb * ell;
        for (int a = threadIdx.x; a < ell; a += blockDim.x) {
            const double t = ck[a];
            ck[a] = cb[a];
            cb[a] = t;
        }
        if (threadIdx.x == 0) {
            double t = nrm[k];
            nrm[k] = nrm[jb];
            nrm[jb] = t;
            t = nrm0[k];
            nrm0[k] = nrm0[jb];
            nrm0[jb] = t;
            const int ti = piv[k];
            piv[k] = piv[jb];
            piv[jb] = ti;
        }
    }
    __syncthreads();
    double s = 0.0;
    for (int a = k + threadIdx.x; a < ell; a += blockDim.x) s += ck[a] * ck[a];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    double tot = 0.0;
    for (int w = 0; w < (int)blockDim.x / 64; ++w) tot += red[w];
    const double alpha = sqrt(tot);
    const double r00 = k == 0 ? alpha : st[1];
    if (threadIdx.x == 0) alphas[k] = alpha;
    if (alpha <= tol * r00) {
        // rank reached: this and the later steps change nothing
        if (threadIdx.x == 0) {
            ist[0] = 1;
            ist[1] = k;
        }
        return;
    }
    const double ckk = ck[k];
    const double beta = ckk > 0 ? -alpha : alpha;
    const double v0 = ckk - beta;
    __syncthreads();
    for (int a = k + 1 + threadIdx.x; a < ell; a += blockDim.x) ck[a] /= v0;
    if (threadIdx.x == 0) {
        st[0] = (beta - ckk) / beta;
        if (k == 0) st[1] = alpha;
        ist[1] = k + 1;
    }
    __syncthreads();
    if (threadIdx.x == 0) ck[k] = beta;
}

// Step k, part 2: apply the reflector to columns k+1..nf-1 (one wave per
// column) and downdate their norms (recomputed when the downdate loses
// accuracy).
__global__ __launch_bounds__(256) void k_qr_update(int k, int nf, int ell, double* __restrict__ Y,
                                                   double* __restrict__ nrm, double* __restrict__ nrm0,
                                                   const double* __restrict__ st, const int* __restrict__ ist) {
    if (ist[0]) return;
    const int j = k + 1 + blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (j >= nf) return;
    const double* ck = Y + (int64_t)k * ell;
    double* cj = Y + (int64_t)j * ell;
    double dot = 0.0;
    for (int a = k + 1 + lane; a < ell; a += 64) dot += ck[a] * cj[a];
    for (int o = 32; o > 0; o >>= 1) dot += __shfl_xor(dot, o, 64);
    dot = (dot + cj[k]) * st[0];
    for (int a = k + 1 + lane; a < ell; a += 64) cj[a] -= dot * ck[a];
    // every lane has read cj[k] above (through dot); one lane writes it
    const double ckj = cj[k] - dot;
    double nn = nrm[j] - ckj * ckj;
    if (nn <= 1e-10 * nrm0[j]) {
        double s = 0.0;
        for (int a = k + 1 + lane; a < ell; a += 64) s += cj[a] * cj[a];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        nn = s;
        if (lane == 0) nrm0[j] = nn;
    }
    if (lane == 0) {
        cj[k] = ckj;
        nrm[j] = nn;
    }
}

// Z = R11^-1 R12: back substitution, one single-wave block per right-hand
// side column (column p + col of Y), z in LDS. R[a][b] = Y[b * ell + a].
__global__ __launch_bounds__(64) void k_trsm_cols(int p, int nrest, int ell, const double* __restrict__ Y,
                                                  double* __restrict__ Z) {
    extern __shared__ double z[];  // p
    const int col = blockIdx.x, lane = threadIdx.x;
    const double* y = Y + (int64_t)(p + col) * ell;
    for (int a = p - 1; a >= 0; --a) {
        double s = 0.0;
        for (int b = a + 1 + lane; b < p; b += 64) s += Y[(int64_t)b * ell + a] * z[b];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) z[a] = (y[a] - s) / Y[(int64_t)a * ell + a];
        __syncthreads();
    }
    for (int a = lane; a < p; a += 64) Z[(int64_t)a * nrest + col] = z[a];
}

// rows of W B in pivot order: WBp[r][k] = wB[piv[r]][k]
__global__ void k_gather_rows(int nf, int K, const int* __restrict__ piv, const double* __restrict__ wB,
                              double* __restrict__ WBp) {
    const int64_t n = (int64_t)nf * K;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = e / K, k = e % K;
        WBp[e] = wB[(int64_t)piv[r] * K + k];
    }
}

// ---------------------------------------------------------------------------
// Batched LU with partial pivoting, one block per system (n x n, row-major,
// in place), then forward and back substitution for nrhs right-hand sides
// (n x nrhs, row-major). Pivot rows are swapped physically.
__global__ __launch_bounds__(256) void k_lu_solve(int n, int nrhs_max, double* __restrict__ A,
                                                  double* __restrict__ F, const int* __restrict__ nrhs,
                                                  int* __restrict__ info) {
    __shared__ double red_v[4];
    __shared__ int red_i[4];
    __shared__ int piv_s;
    const int m = blockIdx.x;
    double* a = A + (int64_t)m * n * n;
    double* f = F + (int64_t)m * n * nrhs_max;
    const int nr = nrhs[m];
    for (int k = 0; k < n; ++k) {
        // pivot: largest |a[i][k]|, i >= k (first on ties)
        double best = -1.0;
        int bi = n;
        for (int i = k + threadIdx.x; i < n; i += blockDim.x) {
            const double v = fabs(a[(int64_t)i * n + k]);
            if (v > best) {
                best = v;
                bi = i;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_down(best, o, 64);
            const int oi = __shfl_down(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (threadIdx.x % 64 == 0) {
            red_v[threadIdx.x / 64] = best;
            red_i[threadIdx.x / 64] = bi;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            int b = 0;
            for (int w = 1; w < 4; ++w)
                if (red_v[w] > red_v[b] || (red_v[w] == red_v[b] && red_i[w] < red_i[b])) b = w;
            piv_s = red_i[b];
            if (!(red_v[b] > 0.0)) info[m] = k + 1;
        }
        __syncthreads();
        const int pr = piv_s;
        if (pr != k && pr < n) {
            for (int c = threadIdx.x; c < n; c += blockDim.x) {
                const double t = a[(int64_t)k * n + c];
                a[(int64_t)k * n + c] = a[(int64_t)pr * n + c];
                a[(int64_t)pr * n + c] = t;
            }
            for (int c = threadIdx.x; c < nr; c += blockDim.x) {
                const double t = f[(int64_t)k * nrhs_max + c];
                f[(int64_t)k * nrhs_max + c] = f[(int64_t)pr * nrhs_max + c];
                f[(int64_t)pr * nrhs_max + c] = t;
            }
        }
        __syncthreads();
        const double d = a[(int64_t)k * n + k];
        // eliminate below the pivot: rows i > k, one row per thread group
        for (int i = k + 1 + threadIdx.x; i < n; i += blockDim.x) {
            const double l = a[(int64_t)i * n + k] / d;
            a[(int64_t)i * n + k] = l;
            for (int c = k + 1; c < n; ++c) a[(int64_t)i * n + c] -= l * a[(int64_t)k * n + c];
            for (int c = 0; c < nr; ++c) f[(int64_t)i * nrhs_max + c] -= l * f[(int64_t)k * nrhs_max + c];
        }
        __syncthreads();
    }
    // back substitution, one thread per right-hand side
    for (int c = threadIdx.x; c < nr; c += blockDim.x)
        for (int i = n - 1; i >= 0; --i) {
            double s = f[(int64_t)i * nrhs_max + c];
            for (int q = i + 1; q < n; ++q) s -= a[(int64_t)i * n + q] * f[(int64_t)q * nrhs_max + c];
            f[(int64_t)i * nrhs_max + c] = s / a[(int64_t)i * n + i];
        }
}


// ---------------------------------------------------------------------------
// Modal kernels G_m(t, t'), m = 0..M (Section 9.1), on the device: G^(1) from
// Legendre functions of the second kind of half-integer degree (complete
// elliptic integrals by the arithmetic-geometric mean, then the upward
// recurrence near chi = 1 or Miller's backward recurrence), G^(2) in closed
// form, G^(3) by composite 20-point Gauss-Legendre rules graded toward phi = 0;
// G_m = G^(1) + s G^(2) - G^(3), s = -1 exterior, +1 interior.
constexpr int kMaxM = 16;

__device__ void elliptic_KE_dev(double kp, double& K, double& E) {
    double a = 1.0, b = kp;
    double sum = 0.5 * (1.0 - kp) * (1.0 + kp);
    double pw = 0.5;
    for (int it = 0; it < 64; ++it) {
        const double c = 0.5 * (a - b);
        const double an = 0.5 * (a + b), bn = sqrt(a * b);
        pw *= 2.0;
        sum += pw * c * c;
        a = an;
        b = bn;
        if (fabs(c) <= 1e-18 * a) break;
    }
    K = M_PI / (2.0 * a);
    E = K * (1.0 - sum);
}

__device__ void toroidal_q_dev(double chim1, int M, double* Q) {
    const double chi = 1.0 + chim1;
    const double k = sqrt(2.0 / (chi + 1.0));
    const double kp = sqrt(chim1 / (chi + 1.0));
    double K, E;
    elliptic_KE_dev(kp, K, E);
    const double q0 = k * K;
    Q[0] = q0;
    if (M == 0) return;
    if (chim1 < 0.01) {
        Q[1] = chi * k * K - (2.0 / k) * E;
        for (int m = 1; m < M; ++m) Q[m + 1] = (2.0 * m * chi * Q[m] - (m - 0.5) * Q[m - 1]) / (m + 0.5);
        return;
    }
    const double r = chi + sqrt(chim1 * (chi + 1.0));
    const int L = M + 12 + (int)ceil(37.0 / log(r));
    double up = 0.0, u = 1e-200;
    for (int m = L; m >= 1; --m) {
        const double dn = (2.0 * m * chi * u - (m + 0.5) * up) / (m - 0.5);
        up = u;
        u = dn;
        if (m - 1 <= M) Q[m - 1] = u;
        if (fabs(u) > 1e200) {
            u *= 1e-200;
            up *= 1e-200;
            for (int j = m - 1; j <= M; ++j) Q[j] *= 1e-200;
        }
    }
    const double f = q0 / Q[0];
    for (int m = 0; m <= M; ++m) Q[m] *= f;
}

__device__ void modal_g3_dev(double A2, double B2, int M, const double* __restrict__ gx,
                             const double* __restrict__ gw, double* out) {
    const double width = 2.0 * sqrt(A2 / B2);
    int L = (int)ceil(log2(M_PI / fmax(width, 1e-300)));
    L = max(2, min(L, 40));
    for (int m = 0; m <= M; ++m) out[m] = 0.0;
    double lo = 0.0;
    for (int j = L; j >= 0; --j) {
        const double hi = M_PI * ldexp(1.0, -j);
        const double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
        for (int q = 0; q < 20; ++q) {
            const double phi = c + h * gx[q];
            const double sp = sin(0.5 * phi);
            const double d = sqrt(A2 + B2 * sp * sp);
            const double f = h * gw[q] * log1p(0.5 * d);
            const double c1 = cos(phi);
            double cm1 = 1.0, cm = c1;
            out[0] += f;
            for (int m = 1; m <= M; ++m) {
                out[m] += f * cm;
                const double cn = 2.0 * c1 * cm - cm1;
                cm1 = cm;
                cm = cn;
            }
        }
        lo = hi;
    }
    for (int m = 0; m <= M; ++m) out[m] /= M_PI;
}

// One thread per quadrature node: Gw[node][m] = wq G_m(t_i, tq).
__global__ void k_modal_nodes(int problem, int M, int64_t nnodes, const int* __restrict__ node_pair,
                              const double* __restrict__ pair_t, const double* __restrict__ tqv,
                              const double* __restrict__ wqv, const double* __restrict__ gx,
                              const double* __restrict__ gw, double* __restrict__ Gw) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnodes) return;
    const double t = pair_t[node_pair[q]], tp = tqv[q];
    const double st = sin(t), stp = sin(tp);
    const double sh = sin(0.5 * (t - tp));
    const double chim1 = fmax(2.0 * sh * sh / (st * stp), 1e-300);
    double Q[kMaxM], g3[kMaxM];
    toroidal_q_dev(chim1, M, Q);
    modal_g3_dev(4.0 * sh * sh, 4.0 * st * stp, M, gx, gw, g3);
    const double t1 = fmin(t, tp), t2 = fmax(t, tp);
    const double ratio = tan(0.5 * t1) / tan(0.5 * t2);
    const double pref = 2.0 / (M_PI * sqrt(st * stp));
    const double s2 = problem == 1 ? -1.0 : 1.0;
    const double w = wqv[q];
    double rp = 1.0;
    for (int m = 0; m <= M; ++m) {
        double g2;
        if (m == 0) {
            g2 = -log(cos(0.5 * t1) * sin(0.5 * t2));
        } else {
            rp *= ratio;
            g2 = rp / (2.0 * m);
        }
        Gw[q * (M + 1) + m] = w * (pref * Q[m] + s2 * g2 - g3[m]);
    }
}

// One block per (i, p) pair: A[m][i][p * order + l] = sum over the pair's nodes
// of Gw[node][m] basis[node][l], in node order.
__global__ __launch_bounds__(256) void k_modal_reduce(int M, int n, int panels, int order,
                                                      const int64_t* __restrict__ pair_ptr,
                                                      const double* __restrict__ basis,
                                                      const double* __restrict__ Gw, double* __restrict__ A) {
    const int pr = blockIdx.x;
    const int i = pr / panels, p = pr % panels;
    const int64_t q0 = pair_ptr[pr], q1 = pair_ptr[pr + 1];
    for (int o = threadIdx.x; o < (M + 1) * order; o += blockDim.x) {
        const int m = o / order, l = o % order;
        double acc = 0.0;
        for (int64_t q = q0; q < q1; ++q) acc += Gw[q * (M + 1) + m] * basis[q * order + l];
        A[((int64_t)m * n + i) * n + (int64_t)p * order + l] = acc;
    }
}
}  // namespace

// ---------------------------------------------------------------------------

GpuFine::GpuFine(hipStream_t s, const std::vector<double>& fxyz_h, const std::vector<double>& wB_h, int K_)
    : stream(s), nf((int)(fxyz_h.size() / 3)), K(K_) {
    chk(hipMalloc((void**)&fxyz, sizeof(double) * fxyz_h.size()), "hipMalloc");
    chk(hipMalloc((void**)&wB, sizeof(double) * wB_h.size()), "hipMalloc");
    chk(hipMemcpyAsync(fxyz, fxyz_h.data(), sizeof(double) * fxyz_h.size(), hipMemcpyHostToDevice, s), "upload");
    chk(hipMemcpyAsync(wB, wB_h.data(), sizeof(double) * wB_h.size(), hipMemcpyHostToDevice, s), "upload");
    chk(hipStreamSynchronize(s), "sync");
}

GpuFine::~GpuFine() {
    if (fxyz) (void)hipFree(fxyz);
    if (wB) (void)hipFree(wB);
}

IdResult interpolative_decomposition_gpu(const GpuFine& fine, int problem, const std::vector<double>& txyz,
                                         double tol_id, int ell0, uint64_t seed) {
    hipStream_t s = fine.stream;
    const int nf = fine.nf, K = fine.K;
    const int nt = (int)(txyz.size() / 3);
    IdResult out;
    Buf<double> dtx(txyz.size());
    dtx.put(txyz, s);
    // A = G(x^t, x^f), nt x nf row-major
    Buf<double> A((size_t)nt * nf);
    hipLaunchKernelGGL(k_green_matrix, dim3((nf + 255) / 256, nt), dim3(256), 0, s, problem, nt, nf, dtx.p,
                       fine.fxyz, A.p, (int64_t)nf);
    chk(hipGetLastError(), "green matrix");
    int ell = std::min(ell0, nt);
    while (true) {
        Buf<double> Om((size_t)ell * nt), Y((size_t)nf * ell), nrm(nf), nrm0(nf), st(2), alphas(ell);
        Buf<int> piv(nf), ist(2);
        hipLaunchKernelGGL(k_gauss, dim3(2048), dim3(256), 0, s, (int64_t)ell * nt, seed + (uint64_t)ell, Om.p);
        chk(hipGetLastError(), "gauss");
        // Y^T (nf x ell, i.e. Y column-major): Y^T[f][a] = sum_t A[t][f] Om[a][t]
        chk(gemm_strided<double>(s, nf, ell, nt, A.p, 1, nf, Om.p, 1, nt, Y.p, ell, 1.0, 0), "sketch gemm");
        hipLaunchKernelGGL(k_colnorms, dim3((nf + 3) / 4), dim3(256), 0, s, nf, ell, Y.p, nrm.p, nrm0.p);
        std::vector<int> iota(nf);
        for (int f = 0; f < nf; ++f) iota[f] = f;
        piv.put(iota, s);
        chk(hipMemsetAsync(ist.p, 0, 2 * sizeof(int), s), "memset");
        chk(hipMemsetAsync(st.p, 0, 2 * sizeof(double), s), "memset");
        const int kmax = std::min(ell, nf);
        for (int k = 0; k < kmax; ++k) {
            hipLaunchKernelGGL(k_qr_pivot, dim3(1), dim3(1024), 0, s, k, nf, ell, tol_id, Y.p, nrm.p, nrm0.p, piv.p,
                               st.p, ist.p, alphas.p);
            if (k + 1 < nf)
                hipLaunchKernelGGL(k_qr_update, dim3((nf - k - 1 + 3) / 4), dim3(256), 0, s, k, nf, ell, Y.p, nrm.p,
                                   nrm0.p, st.p, ist.p);
        }
        chk(hipGetLastError(), "pivoted QR");
        std::vector<int> hist;
        ist.get(hist, s, 2);
        chk(hipStreamSynchronize(s), "sync");
        const int p = hist[1];
        if (!(p < ell - 48 || ell >= nt)) {
            ell = std::min(2 * ell, nt);
            continue;
        }
        if (p < 1) throw std::runtime_error("ID found rank 0");
        out.p = p;
        piv.get(out.piv, s, nf);
        // T = Pi W B = WBp[0:p] + Z WBp[p:nf], Z = R11^-1 R12
        const int nrest = nf - p;
        Buf<double> WBp((size_t)nf * K), Z((size_t)p * std::max(nrest, 1)), T((size_t)p * K);
        hipLaunchKernelGGL(k_gather_rows, dim3(1024), dim3(256), 0, s, nf, K, piv.p, fine.wB, WBp.p);
        chk(hipMemcpyAsync(T.p, WBp.p, sizeof(double) * p * K, hipMemcpyDeviceToDevice, s), "copy");
        if (nrest > 0) {
            hipLaunchKernelGGL(k_trsm_cols, dim3(nrest), dim3(64), sizeof(double) * p, s, p, nrest, ell, Y.p, Z.p);
            chk(hipGetLastError(), "trsm");
            chk(gemm_strided<double>(s, p, K, nrest, Z.p, nrest, 1, WBp.p + (size_t)p * K, K, 1, T.p, K, 1.0, 1),
                "T gemm");
        }
        T.get(out.T, s, (size_t)p * K);
        chk(hipStreamSynchronize(s), "sync");
        out.ell = ell;
        break;
    }
    return out;
}

std::vector<double> field_check_gpu(const GpuFine& fine, int problem, const std::vector<double>& hxyz,
                                    const std::vector<double>& skel_xyz, const std::vector<double>& T) {
    hipStream_t s = fine.stream;
    const int nf = fine.nf, K = fine.K;
    const int nh = (int)(hxyz.size() / 3), p = (int)(skel_xyz.size() / 3);
    Buf<double> dh(hxyz.size()), sx(skel_xyz.size()), dT(T.size()), Gf((size_t)nh * nf), Gs((size_t)nh * p),
        full((size_t)nh * K), sk((size_t)nh * K);
    dh.put(hxyz, s);
    sx.put(skel_xyz, s);
    dT.put(T, s);
    hipLaunchKernelGGL(k_green_matrix, dim3((nf + 255) / 256, nh), dim3(256), 0, s, problem, nh, nf, dh.p, fine.fxyz,
                       Gf.p, (int64_t)nf);
    hipLaunchKernelGGL(k_green_matrix, dim3((p + 255) / 256, nh), dim3(256), 0, s, problem, nh, p, dh.p, sx.p, Gs.p,
                       (int64_t)p);
    chk(hipGetLastError(), "green matrix");
    chk(gemm_strided<double>(s, nh, K, nf, Gf.p, nf, 1, fine.wB, K, 1, full.p, K, 1.0, 0), "check gemm");
    chk(gemm_strided<double>(s, nh, K, p, Gs.p, p, 1, dT.p, K, 1, sk.p, K, 1.0, 0), "check gemm");
    std::vector<double> a, b;
    full.get(a, s, (size_t)nh * K);
    sk.get(b, s, (size_t)nh * K);
    chk(hipStreamSynchronize(s), "sync");
    double maxerr = 0.0, maxval = 0.0;
    for (size_t q = 0; q < a.size(); ++q) {
        maxerr = std::max(maxerr, std::fabs(a[q] - b[q]));
        maxval = std::max(maxval, std::fabs(a[q]));
    }
    return {maxerr, maxval};
}

void modal_solve_gpu(hipStream_t s, int n, int nmodes, std::vector<double>& A, std::vector<double>& F,
                     const std::vector<int>& nrhs, int nrhs_max) {
    Buf<double> dA(A.size()), dF(F.size());
    Buf<int> dn(nrhs.size()), info(nmodes);
    dA.put(A, s);
    dF.put(F, s);
    dn.put(nrhs, s);
    chk(hipMemsetAsync(info.p, 0, sizeof(int) * nmodes, s), "memset");
    hipLaunchKernelGGL(k_lu_solve, dim3(nmodes), dim3(256), 0, s, n, nrhs_max, dA.p, dF.p, dn.p, info.p);
    chk(hipGetLastError(), "batched LU");
    std::vector<int> inf;
    info.get(inf, s, nmodes);
    dF.get(F, s, F.size());
    chk(hipStreamSynchronize(s), "sync");
    for (int m = 0; m < nmodes; ++m)
        if (inf[m]) throw std::runtime_error("singular modal collocation matrix");
}

namespace {

class GpuPrecompute final : public PrecomputeDevice {
public:
    explicit GpuPrecompute(hipStream_t s) : s_(s) {}
    void modal_assemble(int problem, int M, const ModalNodes& nd, std::vector<double>& A) override {
        if (M + 1 > kMaxM) throw std::runtime_error("M too large for the device modal kernels");
        const int64_t nnodes = (int64_t)nd.tq.size();
        const int npairs = (int)nd.pair_t.size();
        const int panels = npairs / nd.n;
        std::vector<int> node_pair((size_t)nnodes);
        for (int pr = 0; pr < npairs; ++pr)
            for (int64_t q = nd.pair_ptr[pr]; q < nd.pair_ptr[pr + 1]; ++q) node_pair[(size_t)q] = pr;
        std::vector<double> gx, gw;
        gauss_legendre(20, gx, gw);
        Buf<int> dnp(node_pair.size());
        Buf<int64_t> dptr(nd.pair_ptr.size());
        Buf<double> dpt(nd.pair_t.size()), dtq(nd.tq.size()), dwq(nd.wq.size()), dbas(nd.basis.size()), dgx(20),
            dgw(20), Gw((size_t)nnodes * (M + 1)), dA((size_t)(M + 1) * nd.n * nd.n);
        dnp.put(node_pair, s_);
        dptr.put(nd.pair_ptr, s_);
        dpt.put(nd.pair_t, s_);
        dtq.put(nd.tq, s_);
        dwq.put(nd.wq, s_);
        dbas.put(nd.basis, s_);
        dgx.put(gx, s_);
        dgw.put(gw, s_);
        hipLaunchKernelGGL(k_modal_nodes, dim3((unsigned)((nnodes + 127) / 128)), dim3(128), 0, s_, problem, M, nnodes,
                           dnp.p, dpt.p, dtq.p, dwq.p, dgx.p, dgw.p, Gw.p);
        chk(hipGetLastError(), "modal kernels");
        hipLaunchKernelGGL(k_modal_reduce, dim3(npairs), dim3(256), 0, s_, M, nd.n, panels, nd.order, dptr.p, dbas.p,
                           Gw.p, dA.p);
        chk(hipGetLastError(), "modal reduction");
        dA.get(A, s_, (size_t)(M + 1) * nd.n * nd.n);
        chk(hipStreamSynchronize(s_), "sync");
    }
    void modal_solve(int nr, int nmodes, std::vector<double>& A, std::vector<double>& F, const std::vector<int>& nrhs,
                     int ncmax) override {
        modal_solve_gpu(s_, nr, nmodes, A, F, nrhs, ncmax);
    }
    void set_fine(const std::vector<double>& fxyz, const std::vector<double>& wB, int K) override {
        fine_.reset();
        fine_ = std::make_unique<GpuFine>(s_, fxyz, wB, K);
    }
    void id(int problem, const std::vector<double>& txyz, double tol_id, int ell0, uint64_t seed, int& p,
            std::vector<int>& piv, std::vector<double>& T) override {
        IdResult r = interpolative_decomposition_gpu(*fine_, problem, txyz, tol_id, ell0, seed);
        p = r.p;
        piv = std::move(r.piv);
        T = std::move(r.T);
    }
    void check(int problem, const std::vector<double>& hxyz, const std::vector<double>& skel_xyz,
               const std::vector<double>& T, double& maxerr, double& maxval) override {
        const std::vector<double> r = field_check_gpu(*fine_, problem, hxyz, skel_xyz, T);
        maxerr = r[0];
        maxval = r[1];
    }

private:
    hipStream_t s_;
    std::unique_ptr<GpuFine> fine_;
};

}  // namespace

std::unique_ptr<PrecomputeDevice> make_gpu_precompute(hipStream_t s) { return std::make_unique<GpuPrecompute>(s); }

}  // namespace nce
