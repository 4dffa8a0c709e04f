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
    // recompressions for targets beyond D_k = 2 eps 2^(k/2), k = 1, 2, ...
    std::vector<FarTable> far;
    // diagnostics of the build
    double id_check = 0;     // held-out far-field error / max field
    int n_train = 0;
};

// Basis order: n ascending, m = -n, -n+2, ..., n (m < 0: sin(|m| theta)).
void zernike_modes(int M, std::vector<int>& n, std::vector<int>& m);
double zernike_radial(int n, int m, double r);

// Build the tables (may take seconds). Throws std::runtime_error on failure.
PatchTables build_tables(int problem, double eps, int M, double tol_id, int nthreads = 0);

// Cache: load/save by key under dir (empty dir = no cache). load returns false if absent.
bool load_tables(const std::string& dir, int problem, double eps, int M, double tol_id,
                 PatchTables& out);
void save_tables(const std::string& dir, const PatchTables& t);

// Quadrature rules (exposed for the host self-tests).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w);

// Modal kernel G_m(t, t'), m = 0..M, of the on-surface Green's function.
void modal_kernel(int problem, double t, double tp, int M, double* out);

}  // namespace nce
