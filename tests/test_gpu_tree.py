"""GPU checks of the hierarchical far field (Sections 7.2-7.3, Section 8 Step 3).

The tree approximates the dense compressed sum; its error is controlled by the
incoming-grid tolerance tol_grid (plus the ID tolerance against the oracle).
Checks: tree vs the GPU's own direct all-pairs sum (same tables, so only the
tree's error remains), tree vs the oracle's sampled rows at the N=1000,
N=10000 (clustered) and N=100000 workloads, FP32 tree vs FP64 tree, and a
tree solve against the direct solve."""
from pathlib import Path

import numpy as np
import pytest

import layouts

pytestmark = pytest.mark.gpu
GOLD = Path(__file__).resolve().parent / "golden"


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


# FP32 applies at grid tolerance 1e-4 and table tolerance 1e-6, the settings
# the 2e-5 bounds on raw FP32 applies below hold for (the library defaults
# are coarser, since the FP32 applies only drive the inner solves; those are
# checked through the mixed solves, which must match the FP64 ones)
FP32_TIGHT = dict(tol_grid_fp32=1e-4, tol_id_fp32=1e-6)


def _rel(y, ref, x):
    return float(np.max(np.abs(y - ref)) / np.max(np.abs(ref - x)))


@pytest.mark.parametrize("layout,N,eps,problem,tol_grid", [
    ("uniform", 2000, 0.005, 0, 1e-8),
    ("uniform", 2000, 0.005, 1, 1e-10),
    ("vmf", 2000, 0.005, 1, 1e-8),
])
def test_tree_matches_direct(torch, layout, N, eps, problem, tol_grid):
    import paper_1906_04209_amd as nce
    c = layouts.uniform_centers(N, eps, 11) if layout == "uniform" else layouts.vmf_centers(N, eps, 12)
    d = nce.Context(c, eps, problem=problem, tol_id=1e-12, far_field=nce.FAR_DIRECT)
    t = nce.Context(c, eps, problem=problem, tol_id=1e-12, tol_grid=tol_grid, far_field=nce.FAR_TREE, **FP32_TIGHT)
    x_np = layouts.random_coeffs(N, d.K, 5, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    yd = d.matvec(x).cpu().numpy()
    yt = t.matvec(x).cpu().numpy()
    err = _rel(yt, yd, x_np)
    print(f"{layout} N={N} problem={problem} tol_grid={tol_grid}: levels {t.levels} work {t.work()} err {err:.3e}")
    assert err < 10 * tol_grid
    ym = t.matvec(x, precision=nce.MIXED).cpu().numpy()
    errm = _rel(ym, yd, x_np)
    # at the library's default FP32 tolerances (grids 3e-4, tables 1e-5): the
    # apply error scales with the grid tolerance (about 0.1 of it)
    td = nce.Context(c, eps, problem=problem, tol_id=1e-12, tol_grid=tol_grid, far_field=nce.FAR_TREE)
    errd = _rel(td.matvec(x, precision=nce.MIXED).cpu().numpy(), yd, x_np)
    print(f"  FP32 tree vs FP64 direct {errm:.3e} (grids 1e-4, tables 1e-6), {errd:.3e} (defaults)")
    assert errm < 2e-5
    assert errd < 1e-4


@pytest.mark.parametrize("name,far", [("cfg2", "tree"), ("cfg3", "tree"), ("cfg5", "tree")])
def test_tree_rows_vs_oracle(torch, name, far):
    import paper_1906_04209_amd as nce
    g = np.load(GOLD / f"{name}_rows.npz")
    cfg = layouts.CONFIGS[name]
    tol_id = float(g["tol_id"]) if "tol_id" in g.files else 1e-12
    c = layouts.config_layout(cfg)
    ctx = nce.Context(c, cfg["eps"], problem=cfg["problem"], tol_id=tol_id, tol_grid=1e-8,
                      far_field=nce.FAR_TREE)
    x_np = layouts.random_coeffs(cfg["N"], ctx.K, 777, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    y = ctx.matvec(x).cpu().numpy()
    rows = g["rows"]
    err = _rel(y[rows], g["y"], x_np[rows])
    print(f"{name}: levels {ctx.levels} work {ctx.work()} rows {len(rows)} err {err:.3e}")
    assert err < 1e-9


def test_tree_solve_matches_direct(torch):
    import paper_1906_04209_amd as nce
    cfg = layouts.CONFIGS["cfg2"]
    c = layouts.config_layout(cfg)
    rd = nce.Context(c, cfg["eps"], problem=0, tol_id=1e-12, far_field=nce.FAR_DIRECT).solve()
    rt = nce.Context(c, cfg["eps"], problem=0, tol_id=1e-12, tol_grid=1e-10, far_field=nce.FAR_TREE).solve()
    rm = nce.Context(c, cfg["eps"], problem=0, tol_id=1e-12, tol_grid=1e-10, far_field=nce.FAR_TREE,
                     precision=nce.MIXED).solve()
    print("mu direct", rd["mu"], rd["iters_fp64"], "tree", rt["mu"], rt["iters_fp64"], "tree mixed", rm["mu"],
          rm["iters_fp32"], rm["outer"])
    assert rd["converged"] and rt["converged"] and rm["converged"]
    assert abs(rt["mu"] - rd["mu"]) < 1e-9 * rd["mu"]
    assert abs(rm["mu"] - rd["mu"]) < 1e-9 * rd["mu"]


def test_autotune_shapes_keep_result(torch):
    """Every kernel shape the autotuner may pick gives the same apply up to
    summation order."""
    import paper_1906_04209_amd as nce
    cfg = layouts.CONFIGS["cfg2"]
    c = layouts.config_layout(cfg)
    ctx = nce.Context(c, cfg["eps"], problem=cfg["problem"], tol_id=1e-11, far_field=nce.FAR_TREE)
    x = torch.from_numpy(layouts.random_coeffs(cfg["N"], ctx.K, 5, decay=0.1)).cuda()
    ref64 = ctx.matvec(x, precision=nce.FP64)
    ref32 = ctx.matvec(x, precision=nce.MIXED)
    ch64 = ctx.autotune(nce.FP64)
    ch32 = ctx.autotune(nce.MIXED)
    y64 = ctx.matvec(x, precision=nce.FP64)
    y32 = ctx.matvec(x, precision=nce.MIXED)
    d = (ref64 - x).abs().max().item()
    e64 = (y64 - ref64).abs().max().item() / d
    e32 = (y32 - ref32).abs().max().item() / d
    print(f"autotune FP64 {ch64} FP32 {ch32}: change FP64 {e64:.2e} FP32 {e32:.2e}")
    assert ch64[0] in (0, 4, 8, 16) and ch64[1] in (2, 4, 8) and ch32[0] in (0, 4, 8, 16) and ch32[1] in (2, 4, 8)
    assert e64 < 1e-13
    assert e32 < 1e-6
    # every P2L form, the matrix-core one included, against the 8-point form
    for pr, tol in ((nce.FP64, 1e-13), (nce.MIXED, 1e-6)):
        ctx.set_shapes(pr, 8, 2)
        ref = ctx.matvec(x, precision=pr)
        for shape in (0, 4, 16):
            ctx.set_shapes(pr, shape, 2)
            e = (ctx.matvec(x, precision=pr) - ref).abs().max().item() / d
            print(f"P2L shape {shape} precision {pr}: change {e:.2e}")
            assert e < tol


@pytest.fixture(scope="module")
def cfg2_onepatch():
    """The oracle's interior one-patch solution and tables at eps = 0.01 (CPU)."""
    from conftest import oracle_onepatch
    cfg = layouts.CONFIGS["cfg2"]
    return oracle_onepatch(cfg["problem"], cfg["eps"])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_cfg2_tree_solution_dirichlet_condition(torch, cfg2_onepatch, precision):
    """The tree-accelerated solve of the N = 1000 interior workload satisfies
    u = 1 on its patches at random off-grid points (single-layer potential of
    the library's densities evaluated by the oracle: the patch's own data plus
    every other patch by fine quadrature), to the tree and ID tolerances."""
    import paper_1906_04209_amd as nce
    from oracle import system
    cfg = layouts.CONFIGS["cfg2"]
    c = layouts.config_layout(cfg)
    tab, op = cfg2_onepatch
    pr = nce.FP64 if precision == "fp64" else nce.MIXED
    ctx = nce.Context(c, cfg["eps"], problem=cfg["problem"], tol_id=1e-11, far_field=nce.FAR_TREE,
                      tol_gmres=1e-10, precision=pr)
    r = ctx.solve()
    assert r["converged"]
    x = r["x"].cpu().numpy().reshape(len(c), ctx.K)
    lay = system.Layout(c, tab)
    g = np.random.default_rng(12)
    worst = 0.0
    for i in g.choice(len(c), 2, replace=False):
        t = cfg["eps"] * np.sqrt(g.random(8))
        th = 2 * np.pi * g.random(8)
        worst = max(worst, float(np.max(np.abs(system.patch_residual(lay, op, x, int(i), t, th)))))
    print(f"cfg2 tree {precision}: max |u - 1| on 2 random patches {worst:.2e}")
    assert worst < 1e-8


def test_cfg3_tree_vs_direct_and_mixed_solve(torch):
    """The clustered exterior workload (N = 10,000, eps = 0.005, vMF layout):
    the tree apply against the GPU's direct all-pairs sum over every row (same
    tables, so the difference is the tree's own error, bounded by tol_grid),
    and the capture rate of the mixed solve (FP32 sums inside FP64
    refinement) against the plain FP64 solve, both to 1e-8, within 1e-6."""
    import paper_1906_04209_amd as nce
    cfg = layouts.CONFIGS["cfg3"]
    c = layouts.config_layout(cfg)
    t = nce.Context(c, cfg["eps"], problem=cfg["problem"], tol_id=1e-11, tol_grid=1e-8, far_field=nce.FAR_TREE,
                    tol_gmres=1e-8)
    d = nce.Context(c, cfg["eps"], problem=cfg["problem"], tol_id=1e-11, far_field=nce.FAR_DIRECT)
    x_np = layouts.random_coeffs(cfg["N"], t.K, 5, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    err = _rel(t.matvec(x).cpu().numpy(), d.matvec(x).cpu().numpy(), x_np)
    d.close()
    print(f"cfg3 tree vs direct over all {cfg['N']} rows: {err:.3e}")
    assert err < 1e-8
    r64 = t.solve(want_coeffs=False, want_flux=False)
    t.set_solver(1e-8, 200, nce.MIXED)
    rm = t.solve(want_coeffs=False, want_flux=False)
    rel = abs(rm["capture_rate"] - r64["capture_rate"]) / r64["capture_rate"]
    print(f"cfg3 capture rate FP64 {r64['capture_rate']:.12f} ({r64['iters_fp64']} applies), mixed "
          f"{rm['capture_rate']:.12f} ({rm['iters_fp32']} FP32 + {rm['iters_fp64']} FP64), rel {rel:.2e}")
    assert r64["converged"] and rm["converged"] and rm["rel_residual"] <= 1e-8
    assert rel < 1e-6
