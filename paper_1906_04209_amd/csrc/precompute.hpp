// Per-eps precompute of the narrow capture / narrow escape solver (host, FP64).
//
// Section 8 Step 1 of Kaye & Greengard: (a) solve the one-patch integral
// equation S B = Q for the scaled Zernike data (Section 9), (b) compress the
// outgoing field of a patch by an interpolative decomposition, T = Pi W B
// (Section 7.1), (c) form I = w^T B (eq. getI). Also the Zernike sampling
// nodes and the discrete transform P (Section 4).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace nce {

// Compressed outgoing representation valid for targets at arclength >= D from
// the source patch centre: p skeleton points (a subset of the fine grid) and
// T (p x K), rho = T f (Section 7.1; Section 8.1 for D > 2 eps).
struct FarTable {
    double D = 0;
    int p = 0;
    std::vector<double> T;                          // p x K
    std::vector<double> skel_t, skel_theta, skel_off;
    double check = 0;
    int n_train = 0;
};

struct PatchTables {
    int problem = 0;     // 0 interior, 1 exterior
    double eps = 0;
    int M = 15;
    int K = 0;           // (M+1)(M+2)/2
    int Kstar = 0;       // (M+1)(2M+2)
    int p = 0;           // skeleton size
    double tol_id = 0;
    // Skeleton and sampling nodes in local polar coordinates (t, theta) about
    // the patch centre, plus the local offset vectors
    //   (cos t - 1, sin t cos theta, sin t sin theta)
    // in the (c, e1, e2) frame, so that x = c + off0 c + off1 e1 + off2 e2.
    std::vector<double> skel_t, skel_theta, skel_off;   // p, p, 3p
    std::vector<double> node_t, node_theta, node_off;   // K*, K*, 3K*
    std::vector<double> T;   // p x K, row-major
    std::vector<double> P;   // K x K*, row-major
    std::vector<double> I;   // K
    // The one-patch densities themselves, for quadrature of a patch's field
    // near it: radial collocation nodes t_l (13 panels x 20), their weights
    // for integrals of sigma over the patch in t (incl. sin t and, on the last
    // panel, the Jacobi factor), and sig[k][l] = the radial profile of basis
    // density k at t_l (density = sig[k][l] times cos(m theta) or sin(|m| theta)).
    std::vector<double> rad_t, rad_w;   // nr, nr
    std::vector<double> sig;            // K x nr, row-major
    // recompressions for targets beyond D_k = 2 eps 2^(k/2), k = 1, 2, ...
    std::vector<FarTable> far;
    double ladder_eps = 0;   // the ladder's radius (eps unless shared with larger patches)
    // diagnostics of the build
    double id_check = 0;     // held-out far-field error / max field
    int n_train = 0;
};

// Basis order: n ascending, m = -n, -n+2, ..., n (m < 0: sin(|m| theta)).
void zernike_modes(int M, std::vector<int>& n, std::vector<int>& m);
double zernike_radial(int n, int m, double r);

// The transform P (K x K*) factors over the sampling grid (M + 1 Gauss-Legendre
// radii x 2M + 2 angles, node q = a (2M + 2) + b) as
//   P[k][q] = rad[k][a] trig[mode[k]][b],
// trig ((2M + 1) x (2M + 2)): rows j = 0..M cos(j theta_b), rows M + m sin(m
// theta_b); rad (K x (M + 1)): the Zernike radial factor with the quadrature
// weights and the normalisation; mode[k] the trig row of basis function k.
void transform_factors(int M, std::vector<double>& trig, std::vector<double>& rad, std::vector<int>& mode);

// Quadrature nodes of the modal collocation integrals (Section 9.2), per
// (target node i, panel p) pair, pair index i * panels + p: nodes
// [pair_ptr[q], pair_ptr[q+1]) at t' = tq with weight wq (2 pi, sin t' and the
// rule folded in) and the panel's `order` basis functions there.
struct ModalNodes {
    int n = 0, order = 0;
    std::vector<double> pair_t;       // target t_i per pair
    std::vector<int64_t> pair_ptr;    // pairs + 1
    std::vector<double> tq, wq;       // per node
    std::vector<double> basis;        // per node x order
};

// Steps of the precompute that may run on a device instead of the host.
struct PrecomputeDevice {
    virtual ~PrecomputeDevice() = default;
    // A[m][i][p * order + l] = sum over the pair's nodes of wq G_m(t_i, tq) basis_l
    // (m = 0..M; A is (M+1) x n x n, row-major)
    virtual void modal_assemble(int problem, int M, const ModalNodes& nodes, std::vector<double>& A) = 0;
    // nmodes systems A_m X = F_m (nr x nr; nr x ncmax, nrhs[m] columns used), F overwritten
    virtual void modal_solve(int nr, int nmodes, std::vector<double>& A, std::vector<double>& F,
                             const std::vector<int>& nrhs, int ncmax) = 0;
    // the fine grid (nf x 3) and W B (nf x K) used by the following calls
    virtual void set_fine(const std::vector<double>& fxyz, const std::vector<double>& wB, int K) = 0;
    // randomized ID of G(x^t, x^f): rank p, column order piv, T = Pi W B (p x K)
    virtual void id(int problem, const std::vector<double>& txyz, double tol_id, int ell0, uint64_t seed, int& p,
                    std::vector<int>& piv, std::vector<double>& T) = 0;
    // outgoing field at held-out points, fine grid vs skeleton: max error and max value
    virtual void check(int problem, const std::vector<double>& hxyz, const std::vector<double>& skel_xyz,
                       const std::vector<double>& T, double& maxerr, double& maxval) = 0;
};

// Build the tables (may take seconds): on the host, or with the modal solves,
// the IDs and their checks on `dev`. Throws std::runtime_error on failure.
// ladder_eps > 0: the recompressions sit at D_k = 2 ladder_eps 2^(k/2) instead
// of 2 eps 2^(k/2) (several patch radii share one ladder, that of the largest).
PatchTables build_tables(int problem, double eps, int M, double tol_id, int nthreads = 0,
                         PrecomputeDevice* dev = nullptr, double ladder_eps = 0.0);

// Cache: load/save by key under dir (empty dir = no cache). load returns false if absent.
bool load_tables(const std::string& dir, int problem, double eps, int M, double tol_id,
                 PatchTables& out, double ladder_eps = 0.0);
void save_tables(const std::string& dir, const PatchTables& t);

// Quadrature rules (exposed for the host self-tests).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w);

// Modal kernel G_m(t, t'), m = 0..M, of the on-surface Green's function.
void modal_kernel(int problem, double t, double tp, int M, double* out);

}  // namespace nce
