// Per-eps precompute (host, FP64): one-patch solver, compressed outgoing
// representation, Zernike transform. See precompute.hpp.
#include "precompute.hpp"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <stdexcept>

namespace nce {

static const double kPi = 3.14159265358979323846;

// ----------------------------------------------------------------------------
// Quadrature: Golub-Welsch eigenvalues of the Jacobi matrix, Newton polish,
// weights from the Christoffel formula.

// Eigenvalues of a symmetric tridiagonal matrix (implicit QL with shifts).
// d: diagonal (n), e: e[i] couples i and i+1 (n, last entry unused).
static void tridiag_eigenvalues(std::vector<double>& d, std::vector<double>& e) {
    const int n = (int)d.size();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        int m;
        do {
            for (m = l; m < n - 1; ++m) {
                double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= 1e-17 * dd) break;
            }
            if (m != l) {
                if (++iter > 200) throw std::runtime_error("tridiagonal QL did not converge");
                double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
                double r = std::hypot(g, 1.0);
                g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
                double s = 1.0, c = 1.0, p = 0.0;
                int i;
                bool early = false;
                for (i = m - 1; i >= l; --i) {
                    double f = s * e[i], b = c * e[i];
                    r = std::hypot(f, g);
                    e[i + 1] = r;
                    if (r == 0.0) {
                        d[i + 1] -= p;
                        e[m] = 0.0;
                        early = true;
                        break;
                    }
                    s = f / r;
                    c = g / r;
                    g = d[i + 1] - p;
                    r = (d[i] - g) * s + 2.0 * c * b;
                    p = s * r;
                    d[i + 1] = g + p;
                    g = c * r - b;
                }
                if (early) continue;
                d[l] -= p;
                e[l] = g;
                e[m] = 0.0;
            }
        } while (m != l);
    }
}

// P_n^{(a,b)}(x) and P_{n-1}^{(a,b)}(x) by the three-term recurrence.
static void jacobi_eval(int n, double a, double b, double x, double& pn, double& pn1) {
    double p0 = 1.0, p1 = 0.5 * ((a - b) + (a + b + 2.0) * x);
    if (n == 0) { pn = p0; pn1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double s = 2.0 * k + a + b;
        double a1 = 2.0 * k * (k + a + b) * (s - 2.0);
        double a2 = (s - 1.0) * (a * a - b * b);
        double a3 = (s - 2.0) * (s - 1.0) * s;
        double a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * s;
        double p2 = ((a2 + a3 * x) * p1 - a4 * p0) / a1;
        p0 = p1;
        p1 = p2;
    }
    pn = p1;
    pn1 = p0;
}

static double jacobi_deriv(int n, double a, double b, double x, double pn, double pn1) {
    double s = 2.0 * n + a + b;
    return (n * ((a - b) - s * x) * pn + 2.0 * (n + a) * (n + b) * pn1) / (s * (1.0 - x * x));
}

void gauss_jacobi(int n, double a, double b, std::vector<double>& x, std::vector<double>& w) {
    std::vector<double> d(n), e(n, 0.0);
    for (int k = 0; k < n; ++k) {
        double s = 2.0 * k + a + b;
        d[k] = (k == 0) ? (b - a) / (a + b + 2.0) : (b * b - a * a) / (s * (s + 2.0));
        if (k + 1 < n) {
            int j = k + 1;
            double sj = 2.0 * j + a + b;
            double bj = 4.0 * j * (j + a) * (j + b) * (j + a + b) /
                        (sj * sj * (sj + 1.0) * (sj - 1.0));
            e[k] = std::sqrt(bj);
        }
    }
    tridiag_eigenvalues(d, e);
    std::sort(d.begin(), d.end());
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double lc = (a + b + 1.0) * std::log(2.0) + std::lgamma(n + a + 1.0) +
                      std::lgamma(n + b + 1.0) - std::lgamma(n + a + b + 1.0) - std::lgamma(n + 1.0);
    for (int i = 0; i < n; ++i) {
        double xi = d[i];
        for (int it = 0; it < 4; ++it) {  // Newton polish
            double pn, pn1;
            jacobi_eval(n, a, b, xi, pn, pn1);
            double dp = jacobi_deriv(n, a, b, xi, pn, pn1);
            double dx = pn / dp;
            xi -= dx;
            if (std::fabs(dx) < 1e-17) break;
        }
        double pn, pn1;
        jacobi_eval(n, a, b, xi, pn, pn1);
        double dp = jacobi_deriv(n, a, b, xi, pn, pn1);
        x[i] = xi;
        w[i] = std::exp(lc) / ((1.0 - xi * xi) * dp * dp);
    }
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
    gauss_jacobi(n, 0.0, 0.0, x, w);
}

// ----------------------------------------------------------------------------
// Zernike basis (Section 4): R_n^m(r) = (-1)^s r^m P_s^{(m,0)}(1 - 2 r^2), s = (n-m)/2.

void zernike_modes(int M, std::vector<int>& n, std::vector<int>& m) {
    n.clear();
    m.clear();
    for (int nn = 0; nn <= M; ++nn)
        for (int mm = -nn; mm <= nn; mm += 2) {
            n.push_back(nn);
            m.push_back(mm);
        }
}

double zernike_radial(int n, int m, double r) {
    m = std::abs(m);
    int s = (n - m) / 2;
    double pn, pn1;
    jacobi_eval(s, (double)m, 0.0, 1.0 - 2.0 * r * r, pn, pn1);
    return ((s & 1) ? -1.0 : 1.0) * std::pow(r, m) * pn;
}

void transform_factors(int M, std::vector<double>& trig, std::vector<double>& rad, std::vector<int>& mode) {
    std::vector<int> zn, zm;
    zernike_modes(M, zn, zm);
    const int K = (int)zn.size(), nth = 2 * M + 2, nrad = M + 1;
    std::vector<double> x, w;
    gauss_legendre(nrad, x, w);
    trig.assign((size_t)(2 * M + 1) * nth, 0.0);
    for (int j = 0; j <= 2 * M; ++j)
        for (int b = 0; b < nth; ++b) {
            const double th = 2.0 * kPi * b / nth;
            trig[(size_t)j * nth + b] = j <= M ? std::cos(j * th) : std::sin((j - M) * th);
        }
    rad.assign((size_t)K * nrad, 0.0);
    mode.assign(K, 0);
    for (int k = 0; k < K; ++k) {
        mode[k] = zm[k] >= 0 ? zm[k] : M - zm[k];
        // orthogonality: the integral of Z_k^2 over the unit disk
        const double nrm = (zm[k] == 0 ? 2.0 : 1.0) * kPi / (2.0 * zn[k] + 2.0);
        for (int a = 0; a < nrad; ++a) {
            const double rho = 0.5 * (x[a] + 1.0), wr = 0.5 * w[a];
            rad[(size_t)k * nrad + a] = zernike_radial(zn[k], zm[k], rho) * rho * wr * (2.0 * kPi / nth) / nrm;
        }
    }
}

// ----------------------------------------------------------------------------
// Modal kernels (Section 9.1).

// Complete elliptic integrals K(k), E(k) by the arithmetic-geometric mean,
// given the complementary modulus k' (accurate as k -> 1).
static void elliptic_KE(double kp, double& K, double& E) {
    double a = 1.0, b = kp;
    double sum = 0.5 * (1.0 - kp) * (1.0 + kp);  // 2^{-1} k^2
    double pw = 0.5;
    for (int it = 0; it < 64; ++it) {
        double c = 0.5 * (a - b);
        double an = 0.5 * (a + b), bn = std::sqrt(a * b);
        pw *= 2.0;
        sum += pw * c * c;
        a = an;
        b = bn;
        if (std::fabs(c) <= 1e-18 * a) break;
    }
    K = kPi / (2.0 * a);
    E = K * (1.0 - sum);
}

// Legendre functions of the second kind of half-integer degree,
// Q[m] = Q_{m-1/2}(chi), m = 0..M, from chi - 1 (passed without cancellation).
// Q_{-1/2} = k K(k) and Q_{1/2} = chi k K(k) - (2/k) E(k) with k^2 = 2/(chi+1);
// upward recurrence close to chi = 1, Miller's backward recurrence otherwise.
static void toroidal_q(double chim1, int M, double* Q) {
    const double chi = 1.0 + chim1;
    const double k = std::sqrt(2.0 / (chi + 1.0));
    const double kp = std::sqrt(chim1 / (chi + 1.0));
    double K, E;
    elliptic_KE(kp, K, E);
    const double q0 = k * K;
    Q[0] = q0;
    if (M == 0) return;
    if (chim1 < 0.01) {
        Q[1] = chi * k * K - (2.0 / k) * E;
        for (int m = 1; m < M; ++m)
            Q[m + 1] = (2.0 * m * chi * Q[m] - (m - 0.5) * Q[m - 1]) / (m + 0.5);
        return;
    }
    const double r = chi + std::sqrt(chim1 * (chi + 1.0));
    const int L = M + 12 + (int)std::ceil(37.0 / std::log(r));
    double up = 0.0, u = 1e-200;  // u_{L+1}, u_L
    for (int m = L; m >= 1; --m) {
        double dn = (2.0 * m * chi * u - (m + 0.5) * up) / (m - 0.5);  // u_{m-1}
        up = u;
        u = dn;
        if (m - 1 <= M) Q[m - 1] = u;
        if (std::fabs(u) > 1e200) {
            u *= 1e-200;
            up *= 1e-200;
            for (int j = m - 1; j <= M; ++j) Q[j] *= 1e-200;
        }
    }
    const double f = q0 / Q[0];
    for (int m = 0; m <= M; ++m) Q[m] *= f;
}

// G^(3)_m = (1/pi) int_0^pi log(1 + d/2) cos(m phi) dphi, composite Gauss-Legendre
// on [0, pi] with breakpoints pi 2^-j graded down to the scale where d varies.
namespace {
struct Rule20 {
    std::vector<double> x, w;
    Rule20() { gauss_legendre(20, x, w); }
};
}  // namespace

static void modal_g3(double A2, double B2, int M, double* out) {
    static const Rule20 rule;  // thread-safe one-time initialisation
    const std::vector<double>& gx = rule.x;
    const std::vector<double>& gw = rule.w;
    double width = 2.0 * std::sqrt(A2 / B2);
    int L = (int)std::ceil(std::log2(kPi / std::max(width, 1e-300)));
    L = std::max(2, std::min(L, 40));
    for (int m = 0; m <= M; ++m) out[m] = 0.0;
    double lo = 0.0;
    for (int j = L; j >= 0; --j) {
        double hi = kPi * std::ldexp(1.0, -j);
        double h = 0.5 * (hi - lo), c = 0.5 * (hi + lo);
        for (int q = 0; q < 20; ++q) {
            double phi = c + h * gx[q];
            double sp = std::sin(0.5 * phi);
            double d = std::sqrt(A2 + B2 * sp * sp);
            double f = h * gw[q] * std::log1p(0.5 * d);
            // cos(m phi) by the Chebyshev recurrence
            double c1 = std::cos(phi), cm1 = 1.0, cm = c1;
            out[0] += f;
            for (int m = 1; m <= M; ++m) {
                out[m] += f * cm;
                double cn = 2.0 * c1 * cm - cm1;
                cm1 = cm;
                cm = cn;
            }
        }
        lo = hi;
    }
    for (int m = 0; m <= M; ++m) out[m] /= kPi;
}

void modal_kernel(int problem, double t, double tp, int M, double* out) {
    double st = std::sin(t), stp = std::sin(tp);
    double sh = std::sin(0.5 * (t - tp));
    double chim1 = std::max(2.0 * sh * sh / (st * stp), 1e-300);
    double Q[64];
    toroidal_q(chim1, M, Q);
    double g3[64];
    modal_g3(4.0 * sh * sh, 4.0 * st * stp, M, g3);
    double t1 = std::min(t, tp), t2 = std::max(t, tp);
    double ratio = std::tan(0.5 * t1) / std::tan(0.5 * t2);
    double pref = 2.0 / (kPi * std::sqrt(st * stp));
    // log(2/d) enters G_E with a minus sign and G_I with a plus sign (Section 2.1).
    double s2 = (problem == 1) ? -1.0 : 1.0;
    double rp = 1.0;
    for (int m = 0; m <= M; ++m) {
        double g1 = pref * Q[m];
        double g2;
        if (m == 0) {
            g2 = -std::log(std::cos(0.5 * t1) * std::sin(0.5 * t2));
        } else {
            rp *= ratio;
            g2 = rp / (2.0 * m);
        }
        out[m] = g1 + s2 * g2 - g3[m];
    }
}

// ----------------------------------------------------------------------------
// Small dense linear algebra.

static void lu_solve_multi(int n, std::vector<double>& A, int nrhs, std::vector<double>& Bm) {
    // A: n x n row-major, B: n x nrhs row-major; partial pivoting.
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = std::fabs(A[(size_t)k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(A[(size_t)i * n + k]) > best) {
                best = std::fabs(A[(size_t)i * n + k]);
                p = i;
            }
        if (best == 0.0) throw std::runtime_error("singular one-patch matrix");
        if (p != k) {
            for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)p * n + j]);
            for (int j = 0; j < nrhs; ++j) std::swap(Bm[(size_t)k * nrhs + j], Bm[(size_t)p * nrhs + j]);
        }
        double inv = 1.0 / A[(size_t)k * n + k];
        for (int i = k + 1; i < n; ++i) {
            double f = A[(size_t)i * n + k] * inv;
            if (f == 0.0) continue;
            for (int j = k + 1; j < n; ++j) A[(size_t)i * n + j] -= f * A[(size_t)k * n + j];
            for (int j = 0; j < nrhs; ++j) Bm[(size_t)i * nrhs + j] -= f * Bm[(size_t)k * nrhs + j];
        }
    }
    for (int j = 0; j < nrhs; ++j)
        for (int i = n - 1; i >= 0; --i) {
            double s = Bm[(size_t)i * nrhs + j];
            for (int k = i + 1; k < n; ++k) s -= A[(size_t)i * n + k] * Bm[(size_t)k * nrhs + j];
            Bm[(size_t)i * nrhs + j] = s / A[(size_t)i * n + i];
        }
}

// ----------------------------------------------------------------------------
// One-patch solver (Section 9.2).

namespace {
constexpr int kPanels = 13;
constexpr int kOrder = 20;
constexpr int kThetaFine = 64;
constexpr int kNout = 24;

struct Radial {
    double eps;
    std::vector<double> br;     // kPanels + 1
    std::vector<double> t;      // kPanels * kOrder
    std::vector<double> wsig;   // radial weight for sigma values
    std::vector<double> xg, wg, xj, wj;  // reference rules
    std::vector<double> lamg, lamj;      // barycentric weights
};

std::vector<double> bary(const std::vector<double>& x) {
    std::vector<double> lam(x.size(), 1.0);
    for (size_t j = 0; j < x.size(); ++j)
        for (size_t k = 0; k < x.size(); ++k)
            if (k != j) lam[j] /= (x[j] - x[k]);
    return lam;
}

void lagrange_row(const std::vector<double>& xn, const std::vector<double>& lam, double x,
                  double* out) {
    const int n = (int)xn.size();
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
        double dx = x - xn[j];
        if (dx == 0.0) {
            for (int k = 0; k < n; ++k) out[k] = (k == j) ? 1.0 : 0.0;
            return;
        }
        out[j] = lam[j] / dx;
        s += out[j];
    }
    for (int j = 0; j < n; ++j) out[j] /= s;
}

Radial make_radial(double eps) {
    Radial R;
    R.eps = eps;
    R.br.push_back(0.0);
    for (int j = 1; j < kPanels; ++j) R.br.push_back((1.0 - std::ldexp(1.0, -j)) * eps);
    R.br.push_back(eps);
    gauss_legendre(kOrder, R.xg, R.wg);
    gauss_jacobi(kOrder, -0.5, 0.0, R.xj, R.wj);
    R.lamg = bary(R.xg);
    R.lamj = bary(R.xj);
    for (int p = 0; p < kPanels; ++p) {
        double lo = R.br[p], hi = R.br[p + 1], h = hi - lo;
        for (int q = 0; q < kOrder; ++q) {
            if (p < kPanels - 1) {
                R.t.push_back(lo + 0.5 * (R.xg[q] + 1.0) * h);
                R.wsig.push_back(0.5 * h * R.wg[q]);
            } else {
                double t = lo + 0.5 * (R.xj[q] + 1.0) * h;
                R.t.push_back(t);
                R.wsig.push_back(std::sqrt(0.5 * h) * R.wj[q] * std::sqrt(eps - t));
            }
        }
    }
    return R;
}

// Subintervals of [lo, hi] bisected until each is no longer than its distance
// to s; s itself is a breakpoint when it lies inside.
void graded(double lo, double hi, double s, std::vector<std::pair<double, double>>& out) {
    out.clear();
    std::vector<std::pair<double, double>> st;
    if (lo < s && s < hi) {
        st.push_back({lo, s});
        st.push_back({s, hi});
    } else {
        st.push_back({lo, hi});
    }
    const double hmin = std::max(1e-15 * (hi - lo), 64.0 * 2.2e-16 * std::max(std::fabs(lo), std::fabs(hi)));
    while (!st.empty()) {
        auto iv = st.back();
        st.pop_back();
        double a = iv.first, b = iv.second;
        double dist = (a <= s && s <= b) ? 0.0 : std::min(std::fabs(s - a), std::fabs(s - b));
        double m = 0.5 * (a + b);
        if ((b - a) <= dist || (b - a) <= hmin || !(a < m && m < b))
            out.push_back(iv);
        else {
            st.push_back({a, m});
            st.push_back({m, b});
        }
    }
}
}  // namespace

// The quadrature nodes of the modal collocation integrals, per (target node i,
// panel p) pair (index i * kPanels + p): the same graded rules as
// assemble_modal, with the weight 2 pi w sin t' (and the Jacobi substitution on
// the last panel) and the panel's Lagrange basis at each node.
static ModalNodes modal_nodes(const Radial& R) {
    const int n = (int)R.t.size();
    ModalNodes out;
    out.n = n;
    out.order = kOrder;
    out.pair_t.resize((size_t)n * kPanels);
    out.pair_ptr.assign(1, 0);
    std::vector<double> xo, wo;
    gauss_legendre(kNout, xo, wo);
    std::vector<std::pair<double, double>> iv;
    std::vector<double> basis(kOrder);
    for (int i = 0; i < n; ++i) {
        const double ti = R.t[i];
        for (int p = 0; p < kPanels; ++p) {
            out.pair_t[(size_t)i * kPanels + p] = ti;
            const double lo = R.br[p], hi = R.br[p + 1], h = hi - lo;
            const bool last = (p == kPanels - 1);
            if (!last) graded(lo, hi, ti, iv);
            else graded(0.0, std::sqrt(h), std::sqrt(R.eps - ti), iv);
            for (auto& ab : iv) {
                const double a = ab.first, b = ab.second, hh = 0.5 * (b - a), c = 0.5 * (a + b);
                for (int q = 0; q < kNout; ++q) {
                    const double u = c + hh * xo[q];
                    double tq, wq;
                    if (!last) {
                        tq = u;
                        wq = hh * wo[q] * std::sin(tq);
                        lagrange_row(R.xg, R.lamg, 2.0 * (tq - lo) / h - 1.0, basis.data());
                    } else {
                        tq = R.eps - u * u;
                        wq = 2.0 * hh * wo[q] * std::sin(tq);
                        lagrange_row(R.xj, R.lamj, 2.0 * (tq - lo) / h - 1.0, basis.data());
                        for (int l = 0; l < kOrder; ++l) basis[l] *= std::sqrt(R.eps - R.t[p * kOrder + l]);
                    }
                    if (tq == ti) continue;
                    out.tq.push_back(tq);
                    out.wq.push_back(2.0 * kPi * wq);
                    out.basis.insert(out.basis.end(), basis.begin(), basis.end());
                }
            }
            out.pair_ptr.push_back((int64_t)out.tq.size());
        }
    }
    return out;
}

// Modal collocation matrices A[m][i][l] (m = 0..M, n = 260).
static void assemble_modal(int problem, const Radial& R, int M, std::vector<double>& A) {
    const int n = (int)R.t.size();
    A.assign((size_t)(M + 1) * n * n, 0.0);
    std::vector<double> xo, wo;
    gauss_legendre(kNout, xo, wo);
#pragma omp parallel
    {
        std::vector<std::pair<double, double>> iv;
        std::vector<double> G(M + 1), basis(kOrder);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < n; ++i) {
            const double ti = R.t[i];
            for (int p = 0; p < kPanels; ++p) {
                const double lo = R.br[p], hi = R.br[p + 1], h = hi - lo;
                const bool last = (p == kPanels - 1);
                if (!last) {
                    graded(lo, hi, ti, iv);
                } else {
                    // in s = sqrt(eps - t'); a target below the panel maps beyond smax
                    double smax = std::sqrt(h);
                    graded(0.0, smax, std::sqrt(R.eps - ti), iv);
                }
                for (auto& ab : iv) {
                    double a = ab.first, b = ab.second, hh = 0.5 * (b - a), c = 0.5 * (a + b);
                    for (int q = 0; q < kNout; ++q) {
                        double u = c + hh * xo[q];
                        double tq, wq;
                        if (!last) {
                            tq = u;
                            wq = hh * wo[q] * std::sin(tq);
                            lagrange_row(R.xg, R.lamg, 2.0 * (tq - lo) / h - 1.0, basis.data());
                        } else {
                            tq = R.eps - u * u;  // t' = eps - s^2, dt' = 2 s ds, sqrt(eps - t') = s
                            wq = 2.0 * hh * wo[q] * std::sin(tq);
                            lagrange_row(R.xj, R.lamj, 2.0 * (tq - lo) / h - 1.0, basis.data());
                            for (int l = 0; l < kOrder; ++l)
                                basis[l] *= std::sqrt(R.eps - R.t[p * kOrder + l]);
                        }
                        // a node that rounds onto the log singularity carries a
                        // weight of a few ulps; dropping it changes nothing
                        if (tq == ti) continue;
                        modal_kernel(problem, ti, tq, M, G.data());
                        for (int m = 0; m <= M; ++m) {
                            double f = 2.0 * kPi * wq * G[m];
                            double* row = &A[((size_t)m * n + i) * n + (size_t)p * kOrder];
                            for (int l = 0; l < kOrder; ++l) row[l] += f * basis[l];
                        }
                    }
                }
            }
        }
    }
}

// ----------------------------------------------------------------------------
// Interpolative decomposition (Section 7.1).

static inline void polar_xyz(double t, double th, double* x) {
    double s = std::sin(t);
    x[0] = s * std::cos(th);
    x[1] = s * std::sin(th);
    x[2] = std::cos(t);
}

static inline double green_surface(int problem, double d) {
    // G_E = 2/d - log(2/d) - log(1 + d/2), G_I = 2/d + log(2/d) - log(1 + d/2)
    double w = 2.0 / d;
    return (problem == 1) ? (w - std::log(w) - std::log1p(0.5 * d))
                          : (w + std::log(w) - std::log1p(0.5 * d));
}

static inline double dist3(const double* a, const double* b) {
    double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
    return std::sqrt(dx * dx + dy * dy + dz * dz);
}

// Training points of the ID for targets at arclength >= D: rings on the
// sphere at Chebyshev radii in dyadic shells from D to pi, 2 kThetaFine
// angles each (n x 3).
static std::vector<double> training_points(double D) {
    std::vector<double> radii;
    const int per = 9;
    double lo = D;
    const double rmax = kPi * (1.0 - 1e-6);
    radii.push_back(lo);
    while (lo < rmax) {
        double hi = std::min(2.0 * lo, rmax);
        for (int q = 1; q <= per; ++q) {
            double x = -std::cos(kPi * q / per);  // Chebyshev-Lobatto, q = 1..per
            radii.push_back(lo + 0.5 * (x + 1.0) * (hi - lo));
        }
        lo = hi;
    }
    const int nth_t = 2 * kThetaFine;
    std::vector<double> txyz(radii.size() * nth_t * 3);
    for (size_t a = 0; a < radii.size(); ++a)
        for (int c = 0; c < nth_t; ++c)
            polar_xyz(radii[a], 2.0 * kPi * c / nth_t, &txyz[((size_t)a * nth_t + c) * 3]);
    return txyz;
}

// 48 held-out points of the region {arclength >= D} (12 on its edge).
static std::vector<double> heldout_points(double D) {
    std::mt19937_64 g2(77);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    const int nh = 48;
    std::vector<double> hx((size_t)3 * nh);
    for (int h = 0; h < nh; ++h) {
        const double r = (h < 12) ? D * (1.0 + 1e-6) : D * std::exp(U(g2) * std::log(kPi / D * 0.999));
        polar_xyz(r, 2.0 * kPi * U(g2), &hx[(size_t)3 * h]);
    }
    return hx;
}

// Skeleton coordinates of the first out.p pivots (fine-grid index l * kThetaFine + c).
static void skeleton_of(FarTable& out, const std::vector<int>& piv, const std::vector<double>& rt) {
    const int p = out.p;
    out.skel_t.resize(p);
    out.skel_theta.resize(p);
    out.skel_off.resize((size_t)3 * p);
    for (int a = 0; a < p; ++a) {
        const int f = piv[a];
        const int l = f / kThetaFine, c = f % kThetaFine;
        const double t = rt[l], th = 2.0 * kPi * c / kThetaFine;
        out.skel_t[a] = t;
        out.skel_theta[a] = th;
        const double sh = std::sin(0.5 * t);
        out.skel_off[3 * a] = -2.0 * sh * sh;
        out.skel_off[3 * a + 1] = std::sin(t) * std::cos(th);
        out.skel_off[3 * a + 2] = std::sin(t) * std::sin(th);
    }
}

// Interpolative decomposition of A = G(x^t, x^f) for training points x^t at
// arclength >= D from the patch centre (Section 7.1): randomized sketch,
// column-pivoted QR, rank by tolerance relative to the largest pivot,
// T = Pi W B and the skeleton (a subset of the fine grid).
static FarTable compress_outgoing(int problem, double D, double tol_id, const std::vector<double>& fxyz,
                                  const std::vector<double>& wB, int K, const std::vector<double>& rt, int ell0,
                                  uint64_t seed, PrecomputeDevice* dev) {
    FarTable out;
    out.D = D;
    const std::vector<double> txyz = training_points(D);
    const int nt = (int)(txyz.size() / 3);
    out.n_train = nt;
    const int nf = (int)(fxyz.size() / 3);
    std::vector<int> piv;
    int p = 0;
    if (dev) {
        dev->id(problem, txyz, tol_id, ell0, seed, p, piv, out.T);
        out.p = p;
        skeleton_of(out, piv, rt);
        const std::vector<double> hx = heldout_points(D);
        std::vector<double> sx((size_t)3 * p);
        for (int a = 0; a < p; ++a)
            for (int d = 0; d < 3; ++d) sx[(size_t)3 * a + d] = fxyz[(size_t)3 * piv[a] + d];
        double maxerr = 0, maxval = 0;
        dev->check(problem, hx, sx, out.T, maxerr, maxval);
        out.check = maxerr / maxval;
        if (!(out.check <= 100.0 * tol_id))
            throw std::runtime_error("compressed outgoing representation failed its held-out check");
        return out;
    }
    int ell = ell0;
    std::vector<double> Rtop;   // p x nf rows of R (column order = piv)
    std::mt19937_64 gen(seed);
    while (true) {
        std::normal_distribution<double> nd(0.0, 1.0);
        std::vector<double> Om((size_t)ell * nt);
        for (auto& v : Om) v = nd(gen);
        // Y = Om A, stored column-major: Y[f * ell + a]
        std::vector<double> Y((size_t)nf * ell, 0.0);
        const int CB = 64;
#pragma omp parallel
        {
            std::vector<double> Ab((size_t)nt * CB);
#pragma omp for schedule(dynamic, 1)
            for (int f0 = 0; f0 < nf; f0 += CB) {
                const int nb = std::min(CB, nf - f0);
                for (int t = 0; t < nt; ++t)
                    for (int j = 0; j < nb; ++j)
                        Ab[(size_t)t * CB + j] = green_surface(problem, dist3(&txyz[(size_t)t * 3], &fxyz[(size_t)(f0 + j) * 3]));
                std::vector<double> acc(CB);
                for (int a = 0; a < ell; ++a) {
                    std::fill(acc.begin(), acc.end(), 0.0);
                    const double* om = &Om[(size_t)a * nt];
                    for (int t = 0; t < nt; ++t) {
                        const double o = om[t];
                        const double* ar = &Ab[(size_t)t * CB];
                        for (int j = 0; j < CB; ++j) acc[j] += o * ar[j];
                    }
                    for (int j = 0; j < nb; ++j) Y[(size_t)(f0 + j) * ell + a] = acc[j];
                }
            }
        }
        // Householder QR with column pivoting on Y (ell x nf, column-major).
        piv.resize(nf);
        for (int f = 0; f < nf; ++f) piv[f] = f;
        std::vector<double> nrm(nf), nrm0(nf);
        for (int f = 0; f < nf; ++f) {
            double s = 0;
            for (int a = 0; a < ell; ++a) s += Y[(size_t)f * ell + a] * Y[(size_t)f * ell + a];
            nrm[f] = nrm0[f] = s;
        }
        double r00 = 0.0;
        p = 0;
        const int kmax = std::min(ell, nf);
        for (int k = 0; k < kmax; ++k) {
            int jb = k;
            for (int j = k + 1; j < nf; ++j)
                if (nrm[j] > nrm[jb]) jb = j;
            if (jb != k) {
                std::swap_ranges(&Y[(size_t)k * ell], &Y[(size_t)k * ell] + ell, &Y[(size_t)jb * ell]);
                std::swap(nrm[k], nrm[jb]);
                std::swap(nrm0[k], nrm0[jb]);
                std::swap(piv[k], piv[jb]);
            }
            double* ck = &Y[(size_t)k * ell];
            double s = 0;
            for (int a = k; a < ell; ++a) s += ck[a] * ck[a];
            double alpha = std::sqrt(s);
            if (k == 0) r00 = alpha;
            if (alpha <= tol_id * r00) break;
            p = k + 1;
            double beta = (ck[k] > 0) ? -alpha : alpha;
            // v = ck[k:] - beta e1, tau = (beta - ck[k]) / beta ... store v in place
            double v0 = ck[k] - beta;
            for (int a = k + 1; a < ell; ++a) ck[a] /= v0;
            const double tau = (beta - ck[k]) / beta;
            ck[k] = beta;
#pragma omp parallel for schedule(static)
            for (int j = k + 1; j < nf; ++j) {
                double* cj = &Y[(size_t)j * ell];
                double dot = cj[k];
                for (int a = k + 1; a < ell; ++a) dot += ck[a] * cj[a];
                dot *= tau;
                cj[k] -= dot;
                for (int a = k + 1; a < ell; ++a) cj[a] -= dot * ck[a];
                double nn = nrm[j] - cj[k] * cj[k];
                if (nn <= 1e-10 * nrm0[j]) {
                    nn = 0.0;
                    for (int a = k + 1; a < ell; ++a) nn += cj[a] * cj[a];
                    nrm0[j] = nn;
                }
                nrm[j] = nn;
            }
        }
        if (p < ell - 48 || ell >= nt) {
            Rtop.assign((size_t)p * nf, 0.0);
            for (int f = 0; f < nf; ++f)
                for (int a = 0; a < p && a <= f; ++a) Rtop[(size_t)a * nf + f] = Y[(size_t)f * ell + a];
            break;
        }
        ell *= 2;
    }
    out.p = p;
    if (p < 1) throw std::runtime_error("ID found rank 0");
    // Pi = [I | R11^-1 R12] in pivot order; T = Pi W B
    out.T.assign((size_t)p * K, 0.0);
    for (int a = 0; a < p; ++a)
        for (int k = 0; k < K; ++k) out.T[(size_t)a * K + k] = wB[(size_t)piv[a] * K + k];
    const int nrest = nf - p;
    // per-thread partial sums, added in thread order afterwards (the same
    // result for a given thread count, whatever the scheduling)
    std::vector<std::vector<double>> Tparts((size_t)omp_get_max_threads());
#pragma omp parallel
    {
        std::vector<double> z(p);
        std::vector<double>& Tloc = Tparts[(size_t)omp_get_thread_num()];
        Tloc.assign((size_t)p * K, 0.0);
#pragma omp for schedule(static)
        for (int j = 0; j < nrest; ++j) {
            const int col = p + j;
            for (int a = p - 1; a >= 0; --a) {
                double s = Rtop[(size_t)a * nf + col];
                for (int b = a + 1; b < p; ++b) s -= Rtop[(size_t)a * nf + b] * z[b];
                z[a] = s / Rtop[(size_t)a * nf + a];
            }
            const double* wb = &wB[(size_t)piv[col] * K];
            for (int a = 0; a < p; ++a) {
                const double za = z[a];
                double* tr = &Tloc[(size_t)a * K];
                for (int k = 0; k < K; ++k) tr[k] += za * wb[k];
            }
        }
    }
    for (const std::vector<double>& Tloc : Tparts)
        for (size_t q = 0; q < Tloc.size(); ++q) out.T[q] += Tloc[q];
    skeleton_of(out, piv, rt);

    // self-check: far field at held-out points of the region, skeleton vs fine grid
    {
        const std::vector<double> hx = heldout_points(D);
        const int nh = (int)(hx.size() / 3);
        double maxerr = 0.0, maxval = 0.0;
        std::vector<double> full(K), sk(K);
        for (int h = 0; h < nh; ++h) {
            const double* x = &hx[(size_t)3 * h];
            std::fill(full.begin(), full.end(), 0.0);
            std::fill(sk.begin(), sk.end(), 0.0);
            for (int f = 0; f < nf; ++f) {
                double gv = green_surface(problem, dist3(x, &fxyz[(size_t)f * 3]));
                for (int k = 0; k < K; ++k) full[k] += gv * wB[(size_t)f * K + k];
            }
            for (int a = 0; a < p; ++a) {
                double gv = green_surface(problem, dist3(x, &fxyz[(size_t)piv[a] * 3]));
                for (int k = 0; k < K; ++k) sk[k] += gv * out.T[(size_t)a * K + k];
            }
            for (int k = 0; k < K; ++k) {
                maxerr = std::max(maxerr, std::fabs(full[k] - sk[k]));
                maxval = std::max(maxval, std::fabs(full[k]));
            }
        }
        out.check = maxerr / maxval;
        if (!(out.check <= 100.0 * tol_id))
            throw std::runtime_error("compressed outgoing representation failed its held-out check");
    }

    return out;
}

PatchTables build_tables(int problem, double eps, int M, double tol_id, int nthreads, PrecomputeDevice* dev,
                         double ladder_eps) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
    PatchTables out;
    out.problem = problem;
    out.eps = eps;
    out.M = M;
    out.tol_id = tol_id;
    if (!(ladder_eps > 0.0)) ladder_eps = eps;
    out.ladder_eps = ladder_eps;
    std::vector<int> zn, zm;
    zernike_modes(M, zn, zm);
    const int K = (int)zn.size();
    out.K = K;

    // (a) one-patch solve
    Radial R = make_radial(eps);
    const int nr = (int)R.t.size();
    std::vector<double> A;
    if (dev) {
        dev->modal_assemble(problem, M, modal_nodes(R), A);
    } else {
        assemble_modal(problem, R, M, A);
    }
    std::vector<double> sigma((size_t)K * nr);
    std::vector<std::vector<int>> cols(M + 1);
    for (int k = 0; k < K; ++k) cols[std::abs(zm[k])].push_back(k);
    if (dev) {
        // all orders at once: A_m (nr x nr) and F_m (nr x ncmax) packed per order
        int ncmax = 0;
        for (const auto& c : cols) ncmax = std::max(ncmax, (int)c.size());
        std::vector<double> F((size_t)(M + 1) * nr * ncmax, 0.0);
        std::vector<int> nrhs(M + 1);
        for (int ma = 0; ma <= M; ++ma) {
            nrhs[ma] = (int)cols[ma].size();
            for (int i = 0; i < nr; ++i)
                for (int c = 0; c < nrhs[ma]; ++c)
                    F[((size_t)ma * nr + i) * ncmax + c] = zernike_radial(zn[cols[ma][c]], ma, R.t[i] / eps);
        }
        dev->modal_solve(nr, M + 1, A, F, nrhs, ncmax);
        for (int ma = 0; ma <= M; ++ma)
            for (int c = 0; c < nrhs[ma]; ++c)
                for (int i = 0; i < nr; ++i)
                    sigma[(size_t)cols[ma][c] * nr + i] = F[((size_t)ma * nr + i) * ncmax + c];
    } else {
        for (int ma = 0; ma <= M; ++ma) {
            std::vector<double> Am(A.begin() + (size_t)ma * nr * nr, A.begin() + (size_t)(ma + 1) * nr * nr);
            const int nc = (int)cols[ma].size();
            std::vector<double> F((size_t)nr * nc);
            for (int i = 0; i < nr; ++i)
                for (int c = 0; c < nc; ++c) F[(size_t)i * nc + c] = zernike_radial(zn[cols[ma][c]], ma, R.t[i] / eps);
            lu_solve_multi(nr, Am, nc, F);
            for (int c = 0; c < nc; ++c)
                for (int i = 0; i < nr; ++i) sigma[(size_t)cols[ma][c] * nr + i] = F[(size_t)i * nc + c];
        }
    }
    // fine grid: radial nodes x kThetaFine angles, index l*kThetaFine + c
    const int nf = nr * kThetaFine;
    std::vector<double> fxyz((size_t)nf * 3), wB((size_t)nf * K), wf(nf);
    for (int l = 0; l < nr; ++l)
        for (int c = 0; c < kThetaFine; ++c) {
            const int f = l * kThetaFine + c;
            const double th = 2.0 * kPi * c / kThetaFine;
            polar_xyz(R.t[l], th, &fxyz[(size_t)f * 3]);
            wf[f] = R.wsig[l] * std::sin(R.t[l]) * (2.0 * kPi / kThetaFine);
            for (int k = 0; k < K; ++k) {
                double ang = zm[k] >= 0 ? std::cos(zm[k] * th) : std::sin(-zm[k] * th);
                wB[(size_t)f * K + k] = wf[f] * sigma[(size_t)k * nr + l] * ang;
            }
        }
    out.rad_t = R.t;
    out.rad_w.resize(nr);
    for (int l = 0; l < nr; ++l) out.rad_w[l] = R.wsig[l] * std::sin(R.t[l]);
    out.sig = sigma;
    // (c) I = w^T B
    out.I.assign(K, 0.0);
    for (int f = 0; f < nf; ++f)
        for (int k = 0; k < K; ++k) out.I[k] += wB[(size_t)f * K + k];

    if (dev) dev->set_fine(fxyz, wB, K);
    // (b) compressed outgoing representation for targets at arclength >= 2 eps
    // (the far-field region of Section 7), then a ladder of recompressions for
    // targets at arclength >= D_k = 2 eps 2^(k/2) (Section 8.1, additional
    // compression of the outgoing representation).
    {
        FarTable base = compress_outgoing(problem, 2.0 * eps, tol_id, fxyz, wB, K, R.t, 384, 0x5eed1234abcdULL, dev);
        out.p = base.p;
        out.T = base.T;
        out.skel_t = base.skel_t;
        out.skel_theta = base.skel_theta;
        out.skel_off = base.skel_off;
        out.id_check = base.check;
        out.n_train = base.n_train;
        int prev = base.p;
        for (int k = 1; k < 40; ++k) {
            const double D = 2.0 * ladder_eps * std::pow(2.0, 0.5 * k);
            if (D > kPi / 3.0) break;
            FarTable ft = compress_outgoing(problem, D, tol_id, fxyz, wB, K, R.t, std::min(384, prev + 64),
                                            0x5eed1234abcdULL + 977 * k, dev);
            prev = ft.p;
            out.far.push_back(std::move(ft));
        }
    }

    // Zernike sampling nodes and transform P (from its two factors)
    {
        std::vector<double> trig, rad;
        std::vector<int> mode;
        transform_factors(M, trig, rad, mode);
        std::vector<double> x, w;
        gauss_legendre(M + 1, x, w);
        const int nth = 2 * M + 2;
        out.Kstar = (M + 1) * nth;
        out.node_t.resize(out.Kstar);
        out.node_theta.resize(out.Kstar);
        out.node_off.resize((size_t)3 * out.Kstar);
        out.P.assign((size_t)K * out.Kstar, 0.0);
        for (int a = 0; a <= M; ++a) {
            const double rho = 0.5 * (x[a] + 1.0);
            for (int b = 0; b < nth; ++b) {
                const int q = a * nth + b;
                const double th = 2.0 * kPi * b / nth, t = eps * rho;
                out.node_t[q] = t;
                out.node_theta[q] = th;
                const double sh = std::sin(0.5 * t);
                out.node_off[3 * q] = -2.0 * sh * sh;
                out.node_off[3 * q + 1] = std::sin(t) * std::cos(th);
                out.node_off[3 * q + 2] = std::sin(t) * std::sin(th);
                for (int k = 0; k < K; ++k)
                    out.P[(size_t)k * out.Kstar + q] = rad[(size_t)k * (M + 1) + a] * trig[(size_t)mode[k] * nth + b];
            }
        }
    }
    for (double v : out.T)
        if (!std::isfinite(v)) throw std::runtime_error("non-finite entry in T");
    if (!(out.I[0] > 0.0) || !std::isfinite(out.I[0])) throw std::runtime_error("bad integral vector");
    return out;
}

// ----------------------------------------------------------------------------
// Cache.

static std::string cache_name(const std::string& dir, int problem, double eps, int M, double tol_id,
                              double ladder_eps) {
    char buf[320];
    if (ladder_eps > 0.0 && ladder_eps != eps)
        std::snprintf(buf, sizeof(buf), "/nce_tables_v3_p%d_eps%.17g_M%d_id%.3g_ladder%.17g.bin", problem, eps, M,
                      tol_id, ladder_eps);
    else
        std::snprintf(buf, sizeof(buf), "/nce_tables_v3_p%d_eps%.17g_M%d_id%.3g.bin", problem, eps, M, tol_id);
    return dir + buf;
}

template <class T>
static void wvec(std::ofstream& f, const std::vector<T>& v) {
    uint64_t n = v.size();
    f.write((const char*)&n, sizeof(n));
    f.write((const char*)v.data(), sizeof(T) * n);
}
template <class T>
static bool rvec(std::ifstream& f, std::vector<T>& v) {
    uint64_t n = 0;
    if (!f.read((char*)&n, sizeof(n))) return false;
    if (n > (1ull << 32)) return false;
    v.resize(n);
    return (bool)f.read((char*)v.data(), sizeof(T) * n);
}

bool load_tables(const std::string& dir, int problem, double eps, int M, double tol_id, PatchTables& t,
                 double ladder_eps) {
    if (dir.empty()) return false;
    std::ifstream f(cache_name(dir, problem, eps, M, tol_id, ladder_eps), std::ios::binary);
    if (!f) return false;
    char magic[8];
    if (!f.read(magic, 8) || std::memcmp(magic, "NCETAB03", 8) != 0) return false;
    int hdr[5];
    double dh[4];
    if (!f.read((char*)hdr, sizeof(hdr)) || !f.read((char*)dh, sizeof(dh))) return false;
    t.problem = hdr[0];
    t.M = hdr[1];
    t.K = hdr[2];
    t.Kstar = hdr[3];
    t.p = hdr[4];
    t.eps = dh[0];
    t.tol_id = dh[1];
    t.id_check = dh[2];
    t.n_train = (int)dh[3];
    bool ok = rvec(f, t.skel_t) && rvec(f, t.skel_theta) && rvec(f, t.skel_off) && rvec(f, t.node_t) &&
              rvec(f, t.node_theta) && rvec(f, t.node_off) && rvec(f, t.T) && rvec(f, t.P) && rvec(f, t.I) &&
              rvec(f, t.rad_t) && rvec(f, t.rad_w) && rvec(f, t.sig);
    uint64_t nfar = 0;
    ok = ok && (bool)f.read((char*)&nfar, sizeof(nfar)) && nfar < 64;
    t.far.assign(ok ? nfar : 0, FarTable());
    for (auto& ft : t.far) {
        double dp[2];
        ok = ok && (bool)f.read((char*)dp, sizeof(dp)) && rvec(f, ft.T) && rvec(f, ft.skel_t) &&
             rvec(f, ft.skel_theta) && rvec(f, ft.skel_off);
        ft.D = dp[0];
        ft.p = (int)dp[1];
        ok = ok && (int)ft.T.size() == ft.p * t.K;
    }
    if (!ok || t.problem != problem || t.M != M || t.eps != eps) return false;
    t.ladder_eps = ladder_eps > 0.0 ? ladder_eps : eps;
    if ((int)t.T.size() != t.p * t.K || (int)t.P.size() != t.K * t.Kstar) return false;
    if (t.rad_w.size() != t.rad_t.size() || t.sig.size() != t.rad_t.size() * (size_t)t.K) return false;
    return true;
}

void save_tables(const std::string& dir, const PatchTables& t) {
    if (dir.empty()) return;
    std::string name = cache_name(dir, t.problem, t.eps, t.M, t.tol_id, t.ladder_eps);
    std::string tmp = name + ".tmp";
    {
        std::ofstream f(tmp, std::ios::binary);
        if (!f) return;
        f.write("NCETAB03", 8);
        int hdr[5] = {t.problem, t.M, t.K, t.Kstar, t.p};
        double dh[4] = {t.eps, t.tol_id, t.id_check, (double)t.n_train};
        f.write((const char*)hdr, sizeof(hdr));
        f.write((const char*)dh, sizeof(dh));
        wvec(f, t.skel_t);
        wvec(f, t.skel_theta);
        wvec(f, t.skel_off);
        wvec(f, t.node_t);
        wvec(f, t.node_theta);
        wvec(f, t.node_off);
        wvec(f, t.T);
        wvec(f, t.P);
        wvec(f, t.I);
        wvec(f, t.rad_t);
        wvec(f, t.rad_w);
        wvec(f, t.sig);
        uint64_t nfar = t.far.size();
        f.write((const char*)&nfar, sizeof(nfar));
        for (const auto& ft : t.far) {
            double dp[2] = {ft.D, (double)ft.p};
            f.write((const char*)dp, sizeof(dp));
            wvec(f, ft.T);
            wvec(f, ft.skel_t);
            wvec(f, ft.skel_theta);
            wvec(f, ft.skel_off);
        }
    }
    std::rename(tmp.c_str(), name.c_str());
}

}  // namespace nce
