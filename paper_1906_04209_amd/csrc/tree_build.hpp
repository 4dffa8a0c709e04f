// Hierarchical far field on a cube-sphere quadtree (Section 7.2 quadtree on
// the sphere, Section 7.3 incoming representations, Section 8 Step 2 and
// Step 3 items 2-4).
//
// Patch centres are projected radially onto the circumscribed cube; each face
// carries a quadtree refined uniformly to the depth L at which no box holds two
// patches (empty boxes pruned). Neighbours are boxes of the same level whose
// closed regions on the cube surface touch, so they wrap across cube edges and
// corners. The interaction list of a box is the set of children of its
// parent's neighbours that are not its own neighbours; at level 0 (the six
// faces, children of the whole sphere) it is the opposite face. For every
// ordered pair of patches the source is then either a level-L neighbour of the
// target or in exactly one interaction list on the target's ancestor path.
//
// A group with interaction-list sources gets an incoming grid -- a
// parity-restricted Chebyshev (radius in [-R, R]) x Fourier (angle) polar grid
// in geodesic polar coordinates about its bounding cap -- when that is cheaper
// than evaluating its sources directly at its members' sampling nodes; sources
// too close to the cap for the grid (or outside the validity region of their
// compressed representation, arclength > 2 eps) are summed directly instead.
// Grid sizes follow from the distance ratio of the closest grid source and the
// grid tolerance.
#pragma once
#include <cstdint>
#include <vector>

#include "precompute.hpp"

namespace nce {

constexpr int kMaxGridQ = 1024;   // grid points per incoming grid (4 per thread x 256)
constexpr int kMaxGridNr = 16;
constexpr int kMaxGridNt = 256;
constexpr int kSrcPerItem = 32;   // source patches per P2L work item (at least)
constexpr size_t kItemPairs = size_t(1) << 18;  // pair evaluations per P2L work item (at least)
constexpr int kLogWindowOctaves = 8;  // binary octaves of the FP64 pair logarithm's argument per P2L item
constexpr int kMaxTableRuns = 8;      // runs of sources sharing one outgoing table per P2L item

struct Tree {
    int nlevels = 0;
    int64_t N = 0;
    // incoming grids
    int ngrid = 0;
    std::vector<double> g_frame;          // ngrid x 9: cap centre, e1, e2
    std::vector<double> g_R;              // cap radius (arclength)
    std::vector<int> g_nr, g_nt, g_level;
    std::vector<int> g_table;             // outgoing table valid at the closest source: 0 = base (D = 2 eps), k = far[k-1]
    std::vector<int64_t> g_off;           // offset of the grid's q values
    std::vector<int> g_item0, g_item1;    // P2L items of the grid
    int64_t total_q = 0;
    // P2L work items: source patches p2l_src[src0 .. src1) onto grid it_grid
    std::vector<int> it_grid, it_src0, it_src1;
    std::vector<int64_t> it_off;          // offset of the item's partial sums
    std::vector<int> p2l_src;
    // the outgoing table of every P2L source (0 = base, k = far[k - 1]): each
    // source's own cheapest table valid over its grid's whole cap; a grid's
    // sources are sorted by it, so an item's sources form at most
    // kMaxTableRuns runs of one table
    std::vector<int> p2l_tab;
    // per item: the first of the kLogWindowOctaves binary octaves that hold the
    // FP64 pair logarithm's argument x of every pair of the item (x in
    // [2^it_win, 2^(it_win + kLogWindowOctaves)), bounded from the geometry)
    std::vector<int> it_win;
    int64_t total_partial = 0;
    // direct lists (near field plus far sources summed directly), CSR over targets
    std::vector<int64_t> dl_ptr;
    std::vector<int> dl_src;
    // grids to interpolate at each patch's sampling nodes, CSR over patches
    std::vector<int64_t> l2t_ptr;
    std::vector<int> l2t_grid;
    // configuration of every item, grid and patch (forest; empty for one tree)
    std::vector<int> it_cfg, g_cfg, pt_cfg;
    // patch type of every item's sources (several patch radii; empty for one)
    std::vector<int> it_type;
    int ncfg = 0;
    // work per matrix-vector product
    double pairs_far = 0, pairs_near = 0, interp_fma = 0;
    int max_q = 0;
};

// Grid size (n_r radial nodes on [0, R], n_theta angles) for a source at
// distance ratio rho = (distance from the cap centre - eps) / R.
void grid_size(double rho, double tol, int& nr, int& nt);

// split_far: a box whose far sources cost less on a second, coarser grid
// gets one (priced with the FP64 kernels' measured rates; the FP32 trees,
// whose small grids gain nothing from it, pass false).
void build_tree(const std::vector<double>& frames, int64_t N, double eps, const PatchTables& tab,
                double tol_grid, Tree& out, bool split_far = true);

// Several patch radii in one configuration: the type of every patch and, per
// (type, outgoing table) with `ntab` tables per type, the first skeleton point
// in the concatenated skeleton offsets, the first strength column in a
// patch's row and the skeleton size; node_stride = entries of a type's
// sampling-node offsets (3 K*).
struct TypeLayout {
    std::vector<int> ptype;
    std::vector<int> t_soff, t_col, t_p;
    int ntab = 1;
    int node_stride = 0;
};

// After build_tree on a layout of several radii (built with the largest radius
// and a common ladder of outgoing-table distances): splits every P2L item so
// that its sources share one type (it_type), and recounts the work with each
// source's own skeleton sizes. frames, eps (the largest radius) and problem as
// for build_tree.
void split_items_by_type(Tree& t, const TypeLayout& tl, int Kstar, const std::vector<double>& frames, double eps,
                         int problem);

// The binary octaves [elo, ehi] of the FP64 pair logarithm's argument (x =
// u^2 + u interior, 1 + 1/u exterior, u half the chord) between the points of
// a grid (within arclength R of its cap centre) and the skeletons of patches
// (within eps of their centres, at arclengths in [dlo, dhi] from the cap
// centre).
void pair_octaves(double dlo, double dhi, double R, double eps, int problem, int& elo, int& ehi);

// A forest: several independent configurations in one patch numbering, each
// contributing its own tree or all-pairs direct lists; the far-field kernels
// then run over every configuration in the same launches.
void start_forest(Tree& t);
// Appends the tree of a configuration whose patches are [first, first + src.N).
void append_tree(Tree& dst, const Tree& src, int64_t first);
// Appends a configuration of n patches starting at `first`, summed directly:
// the direct list of each patch holds every other patch of the configuration.
void append_direct(Tree& dst, int64_t first, int64_t n, int Kstar, int p);
}  // namespace nce
