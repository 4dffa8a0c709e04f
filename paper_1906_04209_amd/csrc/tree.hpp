// Device side of the hierarchical far field (see tree_build.hpp).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "greens.hpp"
#include "tree_build.hpp"

namespace nce {

// The run arrays of a DeviceTree as the P2L kernels take them.
struct TabRuns {
    const int* it_run0;
    const int* run_src;
    const int* run_tab;
};

struct DeviceTree {
    int ngrid = 0, nitems = 0;
    int64_t N = 0;
    int Kstar = 0, p = 0;
    int ptot = 0;              // row length of the strengths (all outgoing tables)
    int* g_table = nullptr;    // per grid: outgoing table index
    int* t_off = nullptr;      // per table: first strength column / skeleton point
    int* t_p = nullptr;        // per table: skeleton size
    double* g_frame = nullptr;
    double* g_T = nullptr;     // per grid: tan(R / 2), its cap radius R in the stereographic radius
    int* g_nr = nullptr;
    int* g_nt = nullptr;
    int64_t* g_off = nullptr;
    int* g_item0 = nullptr;
    int* g_item1 = nullptr;
    int* it_grid = nullptr;
    int* it_src0 = nullptr;
    int* it_src1 = nullptr;
    int64_t* it_off = nullptr;
    int* p2l_src = nullptr;
    int64_t* dl_ptr = nullptr;
    int* dl_src = nullptr;
    int64_t* l2t_ptr = nullptr;
    int* l2t_grid = nullptr;
    // forest: configuration of every item, grid and patch (null for one tree)
    int* it_cfg = nullptr;
    int* g_cfg = nullptr;
    int* pt_cfg = nullptr;
    // several patch radii (null for one): per item its sources' type, per
    // (type, table) the strength column (t_off then gives the skeleton start),
    // per patch its type; node offsets of type t at node_off + t node_stride
    int* it_type = nullptr;
    int* t_col = nullptr;
    int* ptype = nullptr;
    int ntab = 1;
    int node_stride = 0;
    int max_q = 0;
    // half-scaled grid points relative to each cap centre (3 per point, Σq points)
    double* gpt64 = nullptr;
    float* gpt32 = nullptr;
    // items whose grids keep more lanes busy with 4 (resp. 8) grid points per thread
    LogEntry* logtab = nullptr;  // FP64 logarithm table (kLogTab entries)
    // P2L items' sources by outgoing table: item i's runs are [it_run0[i],
    // it_run0[i + 1]); run r starts at source run_src[r] (a place in p2l_src)
    // and uses table run_tab[r] (0 = base, k = far[k - 1])
    int* g_same = nullptr;   // per grid: 1 if its cap (frame and radius) is that of the grid before it
    int* it_run0 = nullptr;
    int* run_src = nullptr;
    int* run_tab = nullptr;
    // the FP64 P2L's logarithm windows: per item its first octave, and the
    // table of octaves win_first .. (kWinBins entries each) they draw from
    int* it_win = nullptr;
    LogEntry* logwin = nullptr;
    int win_first = 0;
    int n_items4 = 0;
    int* items4 = nullptr;
    int* items8 = nullptr;
    // per item: 1 if it is its grid's only item (the P2L block then finishes
    // the grid's coefficients); the grids with several items
    int* it_solo = nullptr;
    int n_multi = 0;
    int* g_multi = nullptr;
    // the transform's trigonometric tables per distinct (nr, nt) and each grid's offset
    double* ttab = nullptr;
    int* g_ttab = nullptr;
    // work buffers (FP64 and FP32)
    double* coef64 = nullptr;
    double* part64 = nullptr;
    float* coef32 = nullptr;
    float* part32 = nullptr;
};

// tab_off / tab_p: offsets and sizes of the outgoing tables in the
// concatenated skeleton and strength arrays (table 0 = base, first).
// tl (several radii, may be null): per-(type, table) skeleton starts,
// strength columns and sizes replace tab_off / tab_p; p is then the largest
// base skeleton.
void upload_tree(const Tree& t, int Kstar, int p, const std::vector<int>& tab_off, const std::vector<int>& tab_p,
                 hipStream_t s, DeviceTree& d, const TypeLayout* tl = nullptr);
void free_tree(DeviceTree& d);

// `live` (may be null): per configuration of a forest, 0 = skip its work in
// this apply (its outputs are then left unspecified).
//
// Step 2: outgoing skeleton sums onto every incoming grid (P2L), reduced per
// grid and turned into Chebyshev-Fourier coefficients.
// r_tgt: grid points per thread of the P2L kernel: 4 (needs max q <= 1024), 8,
// 0 = per item, whichever keeps more lanes busy for its grid, or 16 = the
// matrix-core form (16 x 16 tiles of pair distances on the MFMA units).
template <class T>
hipError_t tree_far(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* skel_off,
                    const T* rho, const int* live = nullptr, int r_tgt = 4);
// Step 3 (direct form): direct-list sums at each patch's sampling nodes; writes U.
template <class T>
hipError_t tree_near(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* node_off,
                     const T* skel_off, const T* rho, T* U, const int* live = nullptr);
// Step 5 fused into step 4 (tree_interp with pa): y_i = x_i + P u_i, u_i the
// patch's node values (near field from U plus the interpolated grids), P
// applied through its factors (transform_factors: trig with its rows zero
// padded to trig_ld, a multiple of 4, rad and mode, as device arrays of the
// apply's precision; M the basis order, K its size). x, y: N x K doubles (may
// alias). U is then read, not written.
template <class T>
struct PApply {
    const T* trig = nullptr;
    int trig_ld = 0;
    const T* rad = nullptr;
    const int* mode = nullptr;
    int M = 0, K = 0;
    const double* x = nullptr;
    double* y = nullptr;
};

// Step 4: interpolate every listed incoming grid at the sampling nodes; adds
// into U, or with pa (non-null) finishes the apply as above.
// npt: sampling nodes per thread (2, 4 or 8 with 256, 128 or 64 threads per patch).
template <class T>
hipError_t tree_interp(hipStream_t s, const DeviceTree& d, const double* frames, const T* node_off, T* U,
                       const int* live = nullptr, int npt = 2, const PApply<T>* pa = nullptr);

}  // namespace nce
