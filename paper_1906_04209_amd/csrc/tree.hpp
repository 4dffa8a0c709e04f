// Hierarchical far field on a cube-sphere quadtree (Section 7.2, 7.3 and
// Section 8 Step 2 and Step 3, items 2-4).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "precompute.hpp"

namespace nce {

struct Tree {
    int nlevels = 0;
    double pairs_far = 0, pairs_near = 0, interp_fma = 0;
};

struct DeviceTree {
    int dummy = 0;
};

void build_tree(const std::vector<double>& frames, int64_t N, double eps, const PatchTables& tab,
                double tol_grid, Tree& out);
void upload_tree(const Tree& t, hipStream_t s, DeviceTree& d);
void free_tree(DeviceTree& d);

// Step 2: outgoing skeleton sums onto every group's incoming grid (P2L).
template <class T>
hipError_t tree_far(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* skel_off,
                    const T* rho);
// Step 3 (direct form): neighbours' skeleton sums at each patch's sampling nodes; writes U.
template <class T>
hipError_t tree_near(hipStream_t s, const DeviceTree& d, int problem, const double* frames, const T* node_off,
                     const T* skel_off, const T* rho, T* U);
// Step 4: interpolate every ancestor group's incoming grid at the sampling nodes; adds into U.
template <class T>
hipError_t tree_interp(hipStream_t s, const DeviceTree& d, const double* frames, const T* node_off, T* U);

}  // namespace nce
