// Host construction of the cube-sphere quadtree, interaction lists, bounding
// caps, incoming-grid sizes and the device work lists (see tree_build.hpp).
#include "tree_build.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <stdexcept>
#include <string>

namespace nce {

namespace {

constexpr int kLmax = 24;  // key resolution per face axis (bits)
constexpr double kPi = 3.14159265358979323846;

uint64_t spread24(uint64_t v) {
    uint64_t r = 0;
    for (int b = 0; b < 24; ++b) r |= ((v >> b) & 1ull) << (2 * b);
    return r;
}

inline double geodesic(const double* a, const double* b) {
    double cr0 = a[1] * b[2] - a[2] * b[1], cr1 = a[2] * b[0] - a[0] * b[2], cr2 = a[0] * b[1] - a[1] * b[0];
    return std::atan2(std::sqrt(cr0 * cr0 + cr1 * cr1 + cr2 * cr2), a[0] * b[0] + a[1] * b[1] + a[2] * b[2]);
}

void frame_of(const double* c, double* f9) {
    double a[3] = {0, 0, 1};
    if (std::fabs(c[2]) > 1.0 / std::sqrt(2.0)) {
        a[0] = 1;
        a[2] = 0;
    }
    double ad = a[0] * c[0] + a[1] * c[1] + a[2] * c[2];
    double e1[3] = {a[0] - ad * c[0], a[1] - ad * c[1], a[2] - ad * c[2]};
    double n = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (double& v : e1) v /= n;
    double e2[3] = {c[1] * e1[2] - c[2] * e1[1], c[2] * e1[0] - c[0] * e1[2], c[0] * e1[1] - c[1] * e1[0]};
    for (int k = 0; k < 3; ++k) {
        f9[k] = c[k];
        f9[3 + k] = e1[k];
        f9[6 + k] = e2[k];
    }
}

struct Box {
    int64_t first, count;  // members: sorted[first .. first+count)
    int face;
    int64_t ix, iy;
    int parent;
    std::vector<int> children;
    std::vector<int> nbrs;
};

// Cuts a grid's run of n sources (their arclengths d from the cap centre, as
// floats; their outgoing tables tb, sorted; skeleton sizes ps) into P2L items
// for a grid of q points: each takes sources until it holds at least
// kSrcPerItem of them and kItemPairs pairs, and ends earlier where its
// tables would form more than kMaxTableRuns runs or its pairs' logarithm
// arguments would leave one window of kLogWindowOctaves octaves. Appends each
// item's end (exclusive) and first octave.
void cut_items(const float* d, const int* tb, const int* ps, size_t n, double q, double R, double eps, int problem,
               std::vector<size_t>& ends, std::vector<int>& first) {
    constexpr double kRel = 1.0 / (1 << 20);  // covers the float rounding of d
    size_t a = 0;
    while (a < n) {
        // the natural end
        size_t b = a;
        int runs = 0;
        double pairs = 0.0;
        while (b < n) {
            if (b == a || tb[b] != tb[b - 1]) {
                if (runs == kMaxTableRuns) break;
                ++runs;
            }
            pairs += q * ps[b];
            ++b;
            if (b - a >= (size_t)kSrcPerItem && pairs >= (double)kItemPairs) break;
        }
        // in one logarithm window (the common case)?
        const auto mm = std::minmax_element(d + a, d + b);
        int lo, hi;
        pair_octaves(*mm.first * (1.0 - kRel), *mm.second * (1.0 + kRel), R, eps, problem, lo, hi);
        if (hi - lo < kLogWindowOctaves) {
            ends.push_back(b);
            first.push_back(lo);
            a = b;
            continue;
        }
        // else the longest prefix that is
        double dmin = d[a], dmax = d[a];
        pair_octaves(dmin * (1.0 - kRel), dmax * (1.0 + kRel), R, eps, problem, lo, hi);
        if (hi - lo >= kLogWindowOctaves) throw std::runtime_error("P2L source beyond one logarithm window");
        size_t e = a + 1;
        while (e < b) {
            if (d[e] < dmin || d[e] > dmax) {
                const double nmin = std::min(dmin, (double)d[e]), nmax = std::max(dmax, (double)d[e]);
                int l, h;
                pair_octaves(nmin * (1.0 - kRel), nmax * (1.0 + kRel), R, eps, problem, l, h);
                if (h - l >= kLogWindowOctaves) break;
                dmin = nmin;
                dmax = nmax;
                lo = l;
            }
            ++e;
        }
        ends.push_back(e);
        first.push_back(lo);
        a = e;
    }
}

// The cheapest outgoing table valid for targets at arclength >= dm from the
// patch centre: 0 = base (valid beyond 2 eps), k = far[k - 1] (beyond D_k);
// among equally cheap ones the first. The valid ladder tables are a prefix
// (the ladder's D increase); its length is first guessed from the ladder's
// spacing D_k = D_1 2^((k-1)/2) by the binary exponent of dm / D_1, then
// corrected against the stored D, so any increasing ladder is chosen exactly.
struct TableChooser {
    std::vector<double> D;
    std::vector<int> best;   // best[c]: the cheapest of tables 0 .. c
    explicit TableChooser(const PatchTables& tab) {
        int b = 0, pb = tab.p;
        best.push_back(0);
        for (size_t k = 0; k < tab.far.size(); ++k) {
            if (k > 0 && !(tab.far[k].D > tab.far[k - 1].D)) throw std::runtime_error("ladder distances not increasing");
            D.push_back(tab.far[k].D);
            if (tab.far[k].p < pb) {
                b = (int)k + 1;
                pb = tab.far[k].p;
            }
            best.push_back(b);
        }
    }
    int operator()(double dm) const {
        const int n = (int)D.size();
        if (n == 0 || !(dm >= D[0])) return 0;
        int e;
        const double m = std::frexp(dm / D[0], &e);   // dm / D_1 = m 2^e, m in [1/2, 1)
        int c = 2 * (e - 1) + (m >= 0.70710678118654752 ? 2 : 1);
        c = std::max(1, std::min(c, n));
        while (c < n && D[c] <= dm) ++c;
        while (c > 1 && D[c - 1] > dm) --c;
        return best[c];
    }
};

}  // namespace

void pair_octaves(double dlo, double dhi, double R, double eps, int problem, int& elo, int& ehi) {
    // every pair's arclength lies in [dlo - R - eps, dhi + R + eps]; the
    // kernel's x carries rounding far below the 2^-20 margin
    const double tlo = std::max(dlo - R - eps, 0.0), thi = std::min(kPi, dhi + R + eps);
    const double ulo = std::sin(0.5 * tlo), uhi = std::sin(0.5 * thi);
    const double xlo = problem == 0 ? ulo * ulo + ulo : 1.0 + 1.0 / uhi;
    const double xhi = problem == 0 ? uhi * uhi + uhi : 1.0 + 1.0 / ulo;
    if (!(xlo > 0.0) || !std::isfinite(xhi)) throw std::runtime_error("P2L pair at zero distance");
    int e;
    std::frexp(xlo * (1.0 - std::ldexp(1.0, -20)), &e);
    elo = e - 1;
    std::frexp(xhi * (1.0 + std::ldexp(1.0, -20)), &e);
    ehi = e - 1;
}

void grid_size(double rho, double tol, int& nr, int& nt) {
    // Fourier modes of a point source at distance rho R decay like rho^-k on the
    // circle of radius R; Chebyshev coefficients in r on [-R, R] decay like
    // (rho + sqrt(rho^2 - 1))^-n. The counts below were checked numerically
    // (a point source of G at ratio rho, interpolated on caps of radius 1e-3 to
    // 0.5) to reach the tolerance relative to the source's maximum on the cap.
    const double lt = std::log(1.0 / tol);
    nt = 2 * (int)std::ceil(lt / std::log(rho));
    const double rb = rho + std::sqrt(rho * rho - 1.0);
    nr = (int)std::ceil(lt / std::log(rb)) / 2 + 1;
}

void build_tree(const std::vector<double>& frames, int64_t N, double eps, const PatchTables& tab, double tol_grid,
                Tree& out, bool split_far) {
    out = Tree();
    out.N = N;
    const int Kstar = tab.Kstar, p = tab.p;
    // smallest accepted distance ratio of a grid's sources: at 3 the grids are
    // about half the size they are at 2 and the few sources pushed to finer
    // levels or direct lists cost less than that saves (a sweep of 2 to 5 over
    // the N = 1e5 layout gave the fewest priced operations at 3, for both the
    // FP64 and the FP32 tolerances: 26 % fewer than at 2)
    const double rho_min = 3.0;
    const double cpair = 40.0;  // one Green's function pair in multiply-add units (cost model only)
    // the split of a grid's sources by distance ratio, priced in interpolation
    // multiply-adds from the measured FP64 rates (0.77 ns per P2L pair, 0.043 ns
    // per interpolation multiply-add, about 100 of them per (node, grid) set-up)
    const double kPairCost = 18.0, kNodeGridCost = 100.0;

    // 1. project to the cube, face-local keys, sort
    std::vector<uint64_t> key(N);
    std::vector<int> face(N);
    std::vector<int64_t> fx(N), fy(N);
    const double scale = std::ldexp(1.0, kLmax);
    for (int64_t i = 0; i < N; ++i) {
        const double* c = &frames[(size_t)i * 9];
        int a = 0;
        for (int k = 1; k < 3; ++k)
            if (std::fabs(c[k]) > std::fabs(c[a])) a = k;
        const int b = (a + 1) % 3, cc = (a + 2) % 3;
        const double u = c[b] / std::fabs(c[a]), v = c[cc] / std::fabs(c[a]);
        face[i] = 2 * a + (c[a] >= 0 ? 0 : 1);
        int64_t ix = (int64_t)std::floor((u + 1.0) * 0.5 * scale), iy = (int64_t)std::floor((v + 1.0) * 0.5 * scale);
        ix = std::min<int64_t>(std::max<int64_t>(ix, 0), (1ll << kLmax) - 1);
        iy = std::min<int64_t>(std::max<int64_t>(iy, 0), (1ll << kLmax) - 1);
        fx[i] = ix;
        fy[i] = iy;
        key[i] = ((uint64_t)face[i] << 48) | spread24((uint64_t)ix) | (spread24((uint64_t)iy) << 1);
    }
    std::vector<int> sorted(N);
    for (int64_t i = 0; i < N; ++i) sorted[i] = (int)i;
    std::sort(sorted.begin(), sorted.end(), [&](int x, int y) { return key[x] < key[y]; });
    // 2. depth: one past the deepest level at which two patches share a box
    int L = 0;
    for (int64_t s = 1; s < N; ++s) {
        const uint64_t k1 = key[sorted[s - 1]], k2 = key[sorted[s]];
        if ((k1 >> 48) != (k2 >> 48)) continue;
        const uint64_t x = (k1 ^ k2) & ((1ull << 48) - 1);
        if (x == 0) throw std::runtime_error("two patch centres project to the same cube point");
        const int h = 63 - __builtin_clzll(x);
        const int common = kLmax - 1 - h / 2;
        L = std::max(L, common + 1);
    }
    if (L > 22) throw std::runtime_error("tree deeper than 22 levels");
    out.nlevels = L + 1;

    // 3. boxes per level (contiguous runs of the sorted order)
    std::vector<std::vector<Box>> lev(L + 1);
    std::vector<std::vector<int>> box_of(L + 1, std::vector<int>(N));  // by sorted position
    for (int l = 0; l <= L; ++l) {
        const int sh = 2 * (kLmax - l);
        int64_t s = 0;
        while (s < N) {
            const uint64_t id = key[sorted[s]] >> sh;
            int64_t e = s + 1;
            while (e < N && (key[sorted[e]] >> sh) == id) ++e;
            Box bx;
            bx.first = s;
            bx.count = e - s;
            const int i0 = sorted[s];
            bx.face = face[i0];
            bx.ix = fx[i0] >> (kLmax - l);
            bx.iy = fy[i0] >> (kLmax - l);
            bx.parent = l > 0 ? box_of[l - 1][s] : -1;
            const int idx = (int)lev[l].size();
            for (int64_t q = s; q < e; ++q) box_of[l][q] = idx;
            if (l > 0) lev[l - 1][bx.parent].children.push_back(idx);
            lev[l].push_back(std::move(bx));
            s = e;
        }
        // neighbours: boxes whose closed regions share a lattice corner on the
        // cube (the four corners of every box, sorted, so that equal corners
        // are adjacent)
        const int64_t S = 1ll << l;
        auto corner = [&](const Box& bx, int di, int dj) {
            const int a = bx.face / 2;
            const int64_t sg = (bx.face % 2 == 0) ? 1 : -1;
            const int b = (a + 1) % 3, cc = (a + 2) % 3;
            std::array<int64_t, 3> P{};
            P[a] = sg * S;
            P[b] = 2 * (bx.ix + di) - S;
            P[cc] = 2 * (bx.iy + dj) - S;
            return P;
        };
        const int nbx = (int)lev[l].size();
        std::vector<std::pair<std::array<int64_t, 3>, int>> cr;
        cr.reserve((size_t)4 * nbx);
        for (int bi = 0; bi < nbx; ++bi)
            for (int di = 0; di < 2; ++di)
                for (int dj = 0; dj < 2; ++dj) cr.emplace_back(corner(lev[l][bi], di, dj), bi);
        std::sort(cr.begin(), cr.end());
        for (size_t a = 0; a < cr.size();) {
            size_t e = a + 1;
            while (e < cr.size() && cr[e].first == cr[a].first) ++e;
            for (size_t x = a; x < e; ++x)
                for (size_t y = a; y < e; ++y)
                    if (cr[x].second != cr[y].second) lev[l][cr[x].second].nbrs.push_back(cr[y].second);
            a = e;
        }
#pragma omp parallel for schedule(static)
        for (int bi = 0; bi < nbx; ++bi) {
            std::vector<int>& nb = lev[l][bi].nbrs;
            std::sort(nb.begin(), nb.end());
            nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        }
    }

    // 4. per patch lists
    std::vector<std::vector<int>> direct(N);
    std::vector<std::vector<int>> l2t(N);
    const double* F = frames.data();
    // grid staging
    std::vector<std::vector<int>> grid_src, grid_tab;   // a grid's sources and their outgoing tables
    // the grid's P2L items: ends in its source list and logarithm windows
    std::vector<std::vector<size_t>> grid_ends;
    std::vector<std::vector<int>> grid_win;
    std::vector<int> ptab(1, p);   // skeleton size per table
    for (const FarTable& ft : tab.far) ptab.push_back(ft.p);
    const TableChooser cheapest_table(tab);

    // One box's far-field work at level l: its interaction list and deferred
    // sources, its bounding cap, which sources its grid takes (sorted by
    // table and cut into items) and which go to its children or to its
    // members' direct lists. Touches only the box's own deferred list, its
    // children's next lists and its members' direct lists, so the boxes of a
    // level run in parallel; the grids are numbered afterwards in box order.
    struct GridOut {
        double f9[9];
        double R = 0;
        int nr = 0, nt = 0, table = 0;
        std::vector<int> src, tab;
        std::vector<size_t> ends;
        std::vector<int> win;
    };
    struct BoxGrid {
        int n = 0;       // grids of the box: 0, 1, or 2 (near sources, far sources)
        GridOut g[2];
    };
    auto process_box = [&](int l, int gi, std::vector<std::vector<int>>& deferred,
                           std::vector<std::vector<int>>& deferred_next, BoxGrid& bg) {
        const Box& g = lev[l][gi];
        // interaction list
        std::vector<int> il;
        if (l == 0) {
            for (int o = 0; o < (int)lev[0].size(); ++o)
                if (o != gi && !std::binary_search(g.nbrs.begin(), g.nbrs.end(), o)) il.push_back(o);
        } else {
            const Box& P = lev[l - 1][g.parent];
            std::vector<int> cand(P.children);
            for (int pn : P.nbrs)
                for (int ch : lev[l - 1][pn].children) cand.push_back(ch);
            for (int o : cand)
                if (o != gi && !std::binary_search(g.nbrs.begin(), g.nbrs.end(), o)) il.push_back(o);
        }
        std::vector<int> src;
        src.swap(deferred[gi]);
        if (il.empty() && src.empty()) return;
        for (int o : il)
            for (int64_t q = lev[l][o].first; q < lev[l][o].first + lev[l][o].count; ++q) src.push_back(sorted[q]);
        // bounding cap of the members' disks (Badoiu-Clarkson iteration, then dilation by eps)
        double cc[3] = {0, 0, 0};
        const int64_t m0 = g.first, mc = g.count;
        for (int64_t q = m0; q < m0 + mc; ++q)
            for (int k = 0; k < 3; ++k) cc[k] += F[(size_t)sorted[q] * 9 + k];
        double nn = std::sqrt(cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2]);
        for (double& v : cc) v /= nn;
        double best[3] = {cc[0], cc[1], cc[2]}, bestR = 1e300;
        if (mc > 1) {
            for (int it = 0; it < 40; ++it) {
                double far = -1;
                int64_t fi = m0;
                for (int64_t q = m0; q < m0 + mc; ++q) {
                    double d = geodesic(cc, &F[(size_t)sorted[q] * 9]);
                    if (d > far) {
                        far = d;
                        fi = q;
                    }
                }
                if (far < bestR) {
                    bestR = far;
                    best[0] = cc[0];
                    best[1] = cc[1];
                    best[2] = cc[2];
                }
                const double* fp = &F[(size_t)sorted[fi] * 9];
                const double t = 1.0 / (it + 2.0);
                for (int k = 0; k < 3; ++k) cc[k] += t * (fp[k] - cc[k]);
                nn = std::sqrt(cc[0] * cc[0] + cc[1] * cc[1] + cc[2] * cc[2]);
                for (double& v : cc) v /= nn;
            }
        } else {
            bestR = 0.0;
            for (int k = 0; k < 3; ++k) best[k] = F[(size_t)sorted[m0] * 9 + k];
        }
        const double R = bestR + eps;
        // sources valid for a grid: the whole cap must lie in the source's
        // far-field region (arclength > 2 eps) and be well separated
        std::vector<int> ok, bad, okt;
        std::vector<float> okd;   // their arclengths from the cap centre
        double rho = 1e300, dmin = 1e300;
        for (int j : src) {
            const double d = geodesic(best, &F[(size_t)j * 9]);
            const double ratio = (d - eps) / R;
            if (d - R > 2.0 * eps * (1.0 + 1e-9) && ratio >= rho_min) {
                ok.push_back(j);
                okd.push_back((float)d);
                // the source's own cheapest table valid over the whole cap
                okt.push_back(cheapest_table(d - R));
                rho = std::min(rho, ratio);
                dmin = std::min(dmin, d - R);
            } else {
                bad.push_back(j);
            }
        }
        bool use_grid = false;
        int nr = 0, nt = 0, table = 0, pt = p;
        if (!ok.empty()) {
            // the table valid at the grid's closest source (the cost model's)
            table = cheapest_table(dmin);
            pt = ptab[table];
            grid_size(rho, tol_grid, nr, nt);
            const double q = (double)nr * nt;
            if (nr <= kMaxGridNr && nt <= kMaxGridNt && q <= kMaxGridQ) {
                const double cost_grid = ok.size() * q * pt * cpair + mc * (double)Kstar * q + q * (nt + 2.0 * nr);
                const double cost_direct = ok.size() * (double)mc * Kstar * p * cpair;
                use_grid = cost_grid < cost_direct;
            }
        }
        if (!use_grid) {
            bad.insert(bad.end(), ok.begin(), ok.end());
            ok.clear();
        }
        if (!bad.empty()) {
            if (l < L) {
                // retry at the children: smaller caps, larger distance ratios
                for (int ch : g.children) {
                    std::vector<int>& dn = deferred_next[ch];
                    dn.insert(dn.end(), bad.begin(), bad.end());
                }
            } else {
                for (int64_t q = m0; q < m0 + mc; ++q) {
                    std::vector<int>& dl = direct[sorted[q]];
                    dl.insert(dl.end(), bad.begin(), bad.end());
                }
            }
        }
        if (!use_grid) return;
        // A second, coarser grid for the far sources where that costs less:
        // the grid is sized by its closest source's distance ratio, so
        // sources at ratio >= tau can share a grid sized for tau instead,
        // at the price of interpolating a second grid at the members' nodes.
        // Priced in interpolation multiply-adds: a P2L pair kPairCost, a
        // grid point per node 1, a (node, grid) set-up kNodeGridCost.
        const size_t n = ok.size();
        double P = 0.0;
        for (int k : okt) P += ptab[k];
        const double q0 = (double)nr * nt, nodes = (double)mc * Kstar;
        double best_cost = kPairCost * q0 * P + nodes * (q0 + kNodeGridCost);
        double tau_best = 0.0;
        int nr_f = 0, nt_f = 0;
        for (double tau : {4.0, 5.0, 6.0, 8.0}) {
            if (!split_far) break;
            double Pn = 0.0, Pf = 0.0, rf = 1e300;
            for (size_t a = 0; a < n; ++a) {
                const double ra = ((double)okd[a] - eps) / R;
                if (ra >= tau) {
                    Pf += ptab[okt[a]];
                    rf = std::min(rf, ra);
                } else {
                    Pn += ptab[okt[a]];
                }
            }
            if (Pn == 0.0 || Pf == 0.0) continue;
            int nrf, ntf;
            grid_size(rf, tol_grid, nrf, ntf);
            const double qf = (double)nrf * ntf;
            const double c = kPairCost * (q0 * Pn + qf * Pf) + nodes * (q0 + qf + 2.0 * kNodeGridCost);
            if (c < best_cost) {
                best_cost = c;
                tau_best = tau;
                nr_f = nrf;
                nt_f = ntf;
            }
        }
        // the grids: sources counting-sorted by table (stable), so that an
        // item's sources form few runs of one table, then cut into items
        auto make_grid = [&](GridOut& go, int gnr, int gnt, bool far_part) {
            frame_of(best, go.f9);
            go.R = R;
            go.nr = gnr;
            go.nt = gnt;
            std::vector<size_t> sel;
            double dm = 1e300;
            for (size_t a = 0; a < n; ++a) {
                const bool is_far = tau_best > 0.0 && ((double)okd[a] - eps) / R >= tau_best;
                if (is_far == far_part) {
                    sel.push_back(a);
                    dm = std::min(dm, (double)okd[a] - R);
                }
            }
            go.table = cheapest_table(dm);
            const size_t m = sel.size();
            std::vector<int> tcount(ptab.size() + 1, 0), pss(m);
            std::vector<float> ds(m);
            for (size_t a : sel) ++tcount[okt[a] + 1];
            for (size_t k = 1; k < tcount.size(); ++k) tcount[k] += tcount[k - 1];
            go.src.resize(m);
            go.tab.resize(m);
            for (size_t a : sel) {
                const int at = tcount[okt[a]]++;
                go.src[at] = ok[a];
                go.tab[at] = okt[a];
                pss[at] = ptab[okt[a]];
                ds[at] = okd[a];
            }
            cut_items(ds.data(), go.tab.data(), pss.data(), m, (double)gnr * gnt, R, eps, tab.problem, go.ends, go.win);
        };
        make_grid(bg.g[0], nr, nt, false);
        bg.n = 1;
        if (tau_best > 0.0) {
            make_grid(bg.g[1], nr_f, nt_f, true);
            bg.n = 2;
        }
    };

    // sources handed down from a parent whose cap was too close to them
    std::vector<std::vector<int>> deferred(lev[0].size()), deferred_next;
    for (int l = 0; l <= L; ++l) {
        if (l < L) deferred_next.assign(lev[l + 1].size(), std::vector<int>());
        const int nb = (int)lev[l].size();
        std::vector<BoxGrid> bgs(nb);
        std::string err;
#pragma omp parallel for schedule(dynamic, 16)
        for (int gi = 0; gi < nb; ++gi) {
            try {
                process_box(l, gi, deferred, deferred_next, bgs[gi]);
            } catch (const std::exception& e) {
#pragma omp critical(tree_build_error)
                if (err.empty()) err = e.what();
            }
        }
        if (!err.empty()) throw std::runtime_error(err);
        // the grids in box order
        for (int gi = 0; gi < nb; ++gi)
            for (int k = 0; k < bgs[gi].n; ++k) {
                GridOut& go = bgs[gi].g[k];
                const int gid = out.ngrid++;
                out.g_frame.insert(out.g_frame.end(), go.f9, go.f9 + 9);
                out.g_R.push_back(go.R);
                out.g_nr.push_back(go.nr);
                out.g_nt.push_back(go.nt);
                out.g_level.push_back(l);
                out.g_table.push_back(go.table);
                grid_src.push_back(std::move(go.src));
                grid_tab.push_back(std::move(go.tab));
                grid_ends.push_back(std::move(go.ends));
                grid_win.push_back(std::move(go.win));
                const Box& g = lev[l][gi];
                for (int64_t q = g.first; q < g.first + g.count; ++q) l2t[sorted[q]].push_back(gid);
            }
        if (l < L) deferred.swap(deferred_next);
    }
    // 5. near field: neighbours at the finest level (one patch per box)
    for (int bi = 0; bi < (int)lev[L].size(); ++bi) {
        const Box& b = lev[L][bi];
        const int i = sorted[b.first];
        for (int o : b.nbrs) {
            const Box& ob = lev[L][o];
            for (int64_t q = ob.first; q < ob.first + ob.count; ++q) direct[i].push_back(sorted[q]);
        }
    }
    // 6. flatten
    out.g_off.resize(out.ngrid);
    out.g_item0.resize(out.ngrid);
    out.g_item1.resize(out.ngrid);
    int64_t qoff = 0, poff = 0;
    for (int g = 0; g < out.ngrid; ++g) {
        const int q = out.g_nr[g] * out.g_nt[g];
        out.max_q = std::max(out.max_q, q);
        out.g_off[g] = qoff;
        qoff += q;
        out.g_item0[g] = (int)out.it_grid.size();
        const std::vector<int>& s = grid_src[g];
        const std::vector<size_t>& ends = grid_ends[g];
        const std::vector<int>& win = grid_win[g];
        for (size_t k = 0, a = 0; k < ends.size(); a = ends[k], ++k) {
            out.it_grid.push_back(g);
            out.it_src0.push_back((int)(out.p2l_src.size() + a));
            out.it_src1.push_back((int)(out.p2l_src.size() + ends[k]));
            out.it_win.push_back(win[k]);
            out.it_off.push_back(poff);
            poff += q;
        }
        out.p2l_src.insert(out.p2l_src.end(), s.begin(), s.end());
        out.p2l_tab.insert(out.p2l_tab.end(), grid_tab[g].begin(), grid_tab[g].end());
        out.g_item1[g] = (int)out.it_grid.size();
        for (int k : grid_tab[g]) out.pairs_far += (double)q * ptab[k];
    }
    out.total_q = qoff;
    out.total_partial = poff;
    out.dl_ptr.assign(N + 1, 0);
    out.l2t_ptr.assign(N + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
        std::sort(direct[i].begin(), direct[i].end());
        out.dl_ptr[i + 1] = out.dl_ptr[i] + (int64_t)direct[i].size();
        out.l2t_ptr[i + 1] = out.l2t_ptr[i] + (int64_t)l2t[i].size();
        out.pairs_near += (double)direct[i].size() * Kstar * p;
        for (int g : l2t[i]) out.interp_fma += (double)Kstar * out.g_nr[g] * out.g_nt[g];
    }
    out.dl_src.reserve(out.dl_ptr[N]);
    out.l2t_grid.reserve(out.l2t_ptr[N]);
    for (int64_t i = 0; i < N; ++i) {
        out.dl_src.insert(out.dl_src.end(), direct[i].begin(), direct[i].end());
        out.l2t_grid.insert(out.l2t_grid.end(), l2t[i].begin(), l2t[i].end());
    }
}

void split_items_by_type(Tree& t, const TypeLayout& tl, int Kstar, const std::vector<double>& frames, double eps,
                         int problem) {
    std::vector<int> it_grid, it_src0, it_src1, it_type, it_win, p2l_src, p2l_tab;
    std::vector<int64_t> it_off;
    int64_t poff = 0;
    t.pairs_far = 0;
    for (int g = 0; g < t.ngrid; ++g) {
        const int q = t.g_nr[g] * t.g_nt[g];
        const int first = t.it_src0[t.g_item0[g]], last = t.it_src1[t.g_item1[g] - 1];
        // the grid's sources, stably grouped by type (each type's keep their
        // order by table)
        std::vector<int> ord((size_t)(last - first));
        for (int a = 0; a < last - first; ++a) ord[a] = first + a;
        std::stable_sort(ord.begin(), ord.end(),
                         [&](int a, int b) { return tl.ptype[t.p2l_src[a]] < tl.ptype[t.p2l_src[b]]; });
        std::vector<int> src(ord.size()), tbs(ord.size()), pss(ord.size());
        std::vector<float> d(ord.size());
        for (size_t a = 0; a < ord.size(); ++a) {
            src[a] = t.p2l_src[ord[a]];
            tbs[a] = t.p2l_tab[ord[a]];
            pss[a] = tl.t_p[tl.ptype[src[a]] * tl.ntab + tbs[a]];
            d[a] = (float)geodesic(&t.g_frame[(size_t)9 * g], &frames[(size_t)src[a] * 9]);
        }
        t.g_item0[g] = (int)it_grid.size();
        size_t a = 0;
        while (a < src.size()) {
            const int ty = tl.ptype[src[a]];
            size_t e = a;
            while (e < src.size() && tl.ptype[src[e]] == ty) ++e;
            std::vector<size_t> ends;
            std::vector<int> win;
            cut_items(d.data() + a, tbs.data() + a, pss.data() + a, e - a, (double)q, t.g_R[g], eps, problem, ends,
                      win);
            for (size_t k = 0, b = a; k < ends.size(); b = a + ends[k], ++k) {
                it_grid.push_back(g);
                it_src0.push_back((int)(p2l_src.size() + b));
                it_src1.push_back((int)(p2l_src.size() + a + ends[k]));
                it_type.push_back(ty);
                it_win.push_back(win[k]);
                it_off.push_back(poff);
                poff += q;
            }
            for (size_t b = a; b < e; ++b) t.pairs_far += (double)q * pss[b];
            a = e;
        }
        p2l_src.insert(p2l_src.end(), src.begin(), src.end());
        p2l_tab.insert(p2l_tab.end(), tbs.begin(), tbs.end());
        t.g_item1[g] = (int)it_grid.size();
    }
    t.it_grid.swap(it_grid);
    t.it_src0.swap(it_src0);
    t.it_src1.swap(it_src1);
    t.it_type.swap(it_type);
    t.it_win.swap(it_win);
    t.it_off.swap(it_off);
    t.p2l_src.swap(p2l_src);
    t.p2l_tab.swap(p2l_tab);
    t.total_partial = poff;
    t.pairs_near = 0;
    for (int64_t i = 0; i < t.N; ++i)
        for (int64_t q = t.dl_ptr[i]; q < t.dl_ptr[i + 1]; ++q)
            t.pairs_near += (double)Kstar * tl.t_p[tl.ptype[t.dl_src[q]] * tl.ntab];
}

void start_forest(Tree& t) {
    t = Tree();
    t.dl_ptr = {0};
    t.l2t_ptr = {0};
}

void append_tree(Tree& dst, const Tree& src, int64_t first) {
    const int g0 = dst.ngrid;
    const int it0 = (int)dst.it_grid.size();
    const int s0 = (int)dst.p2l_src.size();
    const int64_t q0 = dst.total_q, p0 = dst.total_partial;
    dst.nlevels = std::max(dst.nlevels, src.nlevels);
    dst.N += src.N;
    dst.ngrid += src.ngrid;
    dst.g_frame.insert(dst.g_frame.end(), src.g_frame.begin(), src.g_frame.end());
    dst.g_R.insert(dst.g_R.end(), src.g_R.begin(), src.g_R.end());
    dst.g_nr.insert(dst.g_nr.end(), src.g_nr.begin(), src.g_nr.end());
    dst.g_nt.insert(dst.g_nt.end(), src.g_nt.begin(), src.g_nt.end());
    dst.g_level.insert(dst.g_level.end(), src.g_level.begin(), src.g_level.end());
    dst.g_table.insert(dst.g_table.end(), src.g_table.begin(), src.g_table.end());
    for (int g = 0; g < src.ngrid; ++g) {
        dst.g_off.push_back(q0 + src.g_off[g]);
        dst.g_item0.push_back(it0 + src.g_item0[g]);
        dst.g_item1.push_back(it0 + src.g_item1[g]);
    }
    for (size_t it = 0; it < src.it_grid.size(); ++it) {
        dst.it_grid.push_back(g0 + src.it_grid[it]);
        dst.it_src0.push_back(s0 + src.it_src0[it]);
        dst.it_src1.push_back(s0 + src.it_src1[it]);
        dst.it_off.push_back(p0 + src.it_off[it]);
    }
    dst.it_win.insert(dst.it_win.end(), src.it_win.begin(), src.it_win.end());
    for (int j : src.p2l_src) dst.p2l_src.push_back((int)(first + j));
    dst.p2l_tab.insert(dst.p2l_tab.end(), src.p2l_tab.begin(), src.p2l_tab.end());
    dst.it_cfg.insert(dst.it_cfg.end(), src.it_grid.size(), dst.ncfg);
    dst.g_cfg.insert(dst.g_cfg.end(), (size_t)src.ngrid, dst.ncfg);
    dst.pt_cfg.insert(dst.pt_cfg.end(), (size_t)src.N, dst.ncfg);
    dst.ncfg += 1;
    dst.total_q += src.total_q;
    dst.total_partial += src.total_partial;
    for (int64_t i = 0; i < src.N; ++i) {
        dst.dl_ptr.push_back(dst.dl_ptr.back() + (src.dl_ptr[i + 1] - src.dl_ptr[i]));
        dst.l2t_ptr.push_back(dst.l2t_ptr.back() + (src.l2t_ptr[i + 1] - src.l2t_ptr[i]));
    }
    for (int j : src.dl_src) dst.dl_src.push_back((int)(first + j));
    for (int g : src.l2t_grid) dst.l2t_grid.push_back(g0 + g);
    dst.pairs_far += src.pairs_far;
    dst.pairs_near += src.pairs_near;
    dst.interp_fma += src.interp_fma;
    dst.max_q = std::max(dst.max_q, src.max_q);
}

void append_direct(Tree& dst, int64_t first, int64_t n, int Kstar, int p) {
    dst.N += n;
    dst.pt_cfg.insert(dst.pt_cfg.end(), (size_t)n, dst.ncfg);
    dst.ncfg += 1;
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j)
            if (j != i) dst.dl_src.push_back((int)(first + j));
        dst.dl_ptr.push_back(dst.dl_ptr.back() + (n - 1));
        dst.l2t_ptr.push_back(dst.l2t_ptr.back());
    }
    dst.pairs_near += (double)n * (double)(n - 1) * Kstar * (double)p;
}

}  // namespace nce
