"""Several patch radii in one configuration (nce_setup_radii): applies and
solves against the oracle's dense two-radius system (oracle/multitype.py,
goldens by make_golden.py), the tree against the all-pairs sum with two
radii, the absorbing condition on patches of both radii, and the one-radius
case through the same entry point."""
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


def _golden_ctx(problem, **kw):
    import paper_1906_04209_amd as nce
    g = np.load(GOLD / f"mt_p{problem}.npz")
    c, types = layouts.multi_radius_centers(10, g["radii"], int(g["seed"]))
    assert np.array_equal(types, g["types"])
    radius = g["radii"][types]
    kw.setdefault("far_field", nce.FAR_DIRECT)
    return g, c, types, nce.Context(c, radius, problem=problem, tol_id=1e-12, **kw)


@pytest.mark.parametrize("problem", [0, 1])
def test_two_radii_apply_and_solve_vs_oracle(torch, problem):
    import paper_1906_04209_amd as nce
    g, c, types, ctx = _golden_ctx(problem, tol_gmres=1e-12)
    x = layouts.random_coeffs(10, ctx.K, 777, decay=0.1)
    xd = torch.from_numpy(x).cuda()
    ref = g["y"]
    err = np.max(np.abs(ctx.matvec(xd).cpu().numpy() - ref)) / np.max(np.abs(ref - x))
    errm = np.max(np.abs(ctx.matvec(xd, precision=nce.MIXED).cpu().numpy() - ref)) / np.max(np.abs(ref - x))
    key = "mu" if problem == 0 else "capture_rate"
    out = {}
    for name, pr in (("fp64", nce.FP64), ("mixed", nce.MIXED)):
        ctx.set_solver(1e-12, 100, pr)
        r = ctx.solve()
        assert r["converged"]
        rel = abs(r[key] - float(g[key])) / float(g[key])
        ferr = np.max(np.abs(r["flux"].cpu().numpy() - g["flux"])) / np.max(np.abs(g["flux"]))
        xerr = np.max(np.abs(r["x"].cpu().numpy().reshape(10, ctx.K) - g["coeffs"])) / np.max(np.abs(g["coeffs"]))
        out[name] = (rel, ferr, xerr)
    radii, I, t = ctx.types()
    print(f"problem {problem}: radii {radii}, types {t.tolist()}; apply FP64 {err:.2e} FP32 {errm:.2e}; "
          f"(scalar, flux, coefficients) vs oracle {out}")
    # the library numbers radii in ascending order; the patch of each radius is the same
    assert np.allclose(radii, sorted(set(g["radii"].tolist())))
    assert np.array_equal(radii[t], g["radii"][types])
    assert err < 1e-12 and errm < 2e-5
    for rel, ferr, xerr in out.values():
        assert rel < 1e-12 and ferr < 1e-11 and xerr < 1e-11


def test_two_radii_absorbing_condition(torch):
    """The GPU solution meets u = 1 on patches of both radii (the oracle
    evaluates each patch's own data plus every other patch's fine quadrature)."""
    from conftest import oracle_onepatch
    from oracle import multitype
    g, c, types, ctx = _golden_ctx(1, tol_gmres=1e-12)
    r = ctx.solve()
    x = r["x"].cpu().numpy().reshape(10, ctx.K)
    (t0, o0), (t1, o1) = oracle_onepatch(1, float(g["radii"][0])), oracle_onepatch(1, float(g["radii"][1]))
    lay = multitype.Layout(c, types, [t0, t1])
    rng = np.random.default_rng(4)
    worst = 0.0
    for i in range(10):
        eps = float(g["radii"][types[i]])
        t = eps * np.sqrt(rng.random(10))
        th = 2 * np.pi * rng.random(10)
        worst = max(worst, float(np.max(np.abs(multitype.patch_residual(lay, [o0, o1], x, i, t, th)))))
    print(f"two radii: max |u - 1| on the patches {worst:.2e}")
    assert worst < 1e-10


@pytest.mark.parametrize("problem", [0, 1])
def test_two_radii_tree_vs_direct(torch, problem):
    """N = 2000 with radii 0.006 and 0.003: the tree (largest radius's caps and
    ladder, one radius per work item) against the all-pairs sum, FP64 and FP32,
    and the solves through both."""
    import paper_1906_04209_amd as nce
    c, types = layouts.multi_radius_centers(2000, (0.006, 0.003), 61)
    radius = np.array((0.006, 0.003))[types]
    d = nce.Context(c, radius, problem=problem, tol_id=1e-11, far_field=nce.FAR_DIRECT, tol_gmres=1e-10)
    # FP32 at grids 1e-4 and tables 1e-6, the settings of the 2e-5 bound below
    t = nce.Context(c, radius, problem=problem, tol_id=1e-11, tol_grid=1e-8, far_field=nce.FAR_TREE,
                    tol_gmres=1e-10, tol_grid_fp32=1e-4, tol_id_fp32=1e-6)
    x_np = layouts.random_coeffs(2000, d.K, 6, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    yd = d.matvec(x).cpu().numpy()
    yt = t.matvec(x).cpu().numpy()
    err = np.max(np.abs(yt - yd)) / np.max(np.abs(yd - x_np))
    ym = t.matvec(x, precision=nce.MIXED).cpu().numpy()
    errm = np.max(np.abs(ym - yd)) / np.max(np.abs(yd - x_np))
    key = "mu" if problem == 0 else "capture_rate"
    rd, rt = d.solve(want_coeffs=False), t.solve(want_coeffs=False)
    t.set_solver(1e-10, 100, nce.MIXED)
    rm = t.solve(want_coeffs=False)
    print(f"problem {problem}: levels {t.levels} work {t.work()}; tree vs direct {err:.2e}, FP32 tree {errm:.2e}; "
          f"{key} direct {rd[key]:.12f} tree {rt[key]:.12f} mixed {rm[key]:.12f}")
    assert err < 1e-8 and errm < 2e-5
    assert rd["converged"] and rt["converged"] and rm["converged"]
    assert abs(rt[key] - rd[key]) < 1e-9 * abs(rd[key]) and abs(rm[key] - rd[key]) < 1e-8 * abs(rd[key])


def test_one_radius_through_radii_entry(torch):
    import paper_1906_04209_amd as nce
    c = layouts.uniform_centers(30, 0.05, 9)
    a = nce.Context(c, 0.05, problem=1, tol_id=1e-12, far_field=nce.FAR_DIRECT)
    b = nce.Context(c, np.full(30, 0.05), problem=1, tol_id=1e-12, far_field=nce.FAR_DIRECT)
    x = torch.from_numpy(layouts.random_coeffs(30, a.K, 3, decay=0.1)).cuda()
    assert torch.equal(a.matvec(x), b.matvec(x))


@pytest.mark.parametrize("problem", [0, 1])
def test_two_radii_field_vs_oracle(torch, problem):
    """nce_field and nce_patch_residual with two radii, for the oracle's dense
    solution: the potential at points eps_j/5 off patches of both radii, on
    them, on and near the reflecting surface and deep in the domain against
    the oracle's quadrature of every patch; eq. l2res on a patch of each
    radius at the discretisation level, and a 1e-6 change of one coefficient
    raising it."""
    g, c, types, ctx = _golden_ctx(problem)
    x = torch.from_numpy(np.ascontiguousarray(g["coeffs"])).cuda()
    pts = torch.from_numpy(np.ascontiguousarray(g["field_points"])).cuda()
    v = ctx.field(x, pts).cpu().numpy()
    ref = g["field_values"]
    err = np.max(np.abs(v - ref)) / np.max(np.abs(ref))
    res = ctx.patch_residual(x, g["residual_patches"], n_t=6, n_theta=10)
    xp = x.clone()
    xp[0, 0] *= 1 + 1e-6
    resp = ctx.patch_residual(xp, g["residual_patches"][:1], n_t=6, n_theta=10)
    # the physical field (interior: I_sigma over the patches of both radii)
    phys = ctx.field(x, pts, physical=True).cpu().numpy()
    P = g["field_points"]
    if problem == 0:
        want = (ref - 1.0) / (-3.0 * float(g["I_sigma"])) + (1.0 - np.sum(P * P, axis=1)) / 6.0
    else:
        want = 1.0 - ref
    perr = np.max(np.abs(phys - want)) / np.max(np.abs(want))
    print(f"problem {problem}: field vs oracle {err:.2e} over {len(ref)} points, physical {perr:.2e}; residual "
          f"{res} (oracle {g['residual_values']}), perturbed {resp}")
    assert err < 1e-12 and perr < 1e-12
    assert np.all(res < 1e-12)
    assert resp[0] > 100 * res[0]


def _oracle_chi0(problem, eps):
    """Total charge of e_0 in the oracle's stored outgoing table of one radius."""
    from oracle import tables
    t = tables.load(tables.GOLDEN_DIR / (tables.key(problem, eps, 15, 1e-12) + ".npz"))
    return float(t.T[:, 0].sum())


@pytest.mark.parametrize("problem,radii,seed", [(0, (0.01, 0.05), 71), (1, (0.005, 0.05), 72)])
def test_two_radii_coarse_solve_and_deflation_matrix(torch, problem, radii, seed):
    """The coarse model with two radii (ratio 5 and 10), N = 300: each radius's
    charge chi0 against the oracle's outgoing table of that radius, the coarse
    solve satisfying a_i + sum_{j != i} G(c_i, c_j) chi0_j a_j = 1 with the
    closed-form G and the oracle's charges, and the deflation's coarse matrix
    against I + Z^T G D Z, D = diag(chi0_j)."""
    import paper_1906_04209_amd as nce
    from oracle import greens
    from test_host_deflate import harmonic_polys, mgs
    N = 300
    c, types = layouts.multi_radius_centers(N, radii, seed)
    radius = np.asarray(radii)[types]
    ctx = nce.Context(c, radius, problem=problem, tol_id=1e-11, tol_coarse=1e-6)
    a, iters, chi0 = ctx.coarse(with_chi0=True)
    a = a.cpu().numpy()
    lr, _, lt = ctx.types()
    assert np.allclose(lr, sorted(radii))
    want = np.array([_oracle_chi0(problem, float(e)) for e in lr])
    cerr = float(np.max(np.abs(chi0 - want) / np.abs(want)))
    q = want[lt]   # every patch's charge, caller's order
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=-1)
    np.fill_diagonal(d, 1.0)
    G = greens.g_surface(d, problem)
    np.fill_diagonal(G, 0.0)
    res = np.linalg.norm(a + G @ (q * a) - 1.0) / np.sqrt(N)
    # one common charge instead (the largest radius's) misses the equations
    res1 = np.linalg.norm(a + want[-1] * (G @ a) - 1.0) / np.sqrt(N)
    k, T = ctx.deflation_matrix()
    Z = mgs(harmonic_polys(c))
    ref = np.eye(16) + Z.T @ G @ (q[:, None] * Z)
    terr = np.max(np.abs(T - ref)) / np.max(np.abs(ref - np.eye(16)))
    print(f"problem {problem} radii {lr}: chi0 {chi0} (oracle rel err {cerr:.2e}); coarse {iters} iterations, "
          f"residual {res:.2e} (one charge: {res1:.2e}); deflation matrix k {k} rel err {terr:.2e}")
    assert cerr < 1e-9
    assert iters >= 1 and res < 1e-5 and res1 > 100 * res
    assert k == 16 and terr < 1e-5


@pytest.mark.parametrize("problem", [0, 1])
def test_two_radii_deflation_and_coarse_start_keep_result(torch, problem):
    """Mixed solves of N = 3000 patches of radii 0.01 and 0.005 without and
    with the deflation, then with the coarse start as well: the same scalar
    to 1e-8, fewer FP32 applies with the deflation, and a coarse start that
    halves the initial residual at least; the FP64 solve from the coarse start
    gives the same scalar as well."""
    import paper_1906_04209_amd as nce
    c, types = layouts.multi_radius_centers(3000, (0.01, 0.005), 73)
    radius = np.array((0.01, 0.005))[types]
    key = "mu" if problem == 0 else "capture_rate"
    ctx = nce.Context(c, radius, problem=problem, tol_id=1e-11, tol_gmres=1e-10, precision=nce.MIXED,
                      deflation=False)
    out = {"plain": ctx.solve(want_coeffs=False, want_flux=False)}
    ctx.set_deflation(True)
    out["deflated"] = ctx.solve(want_coeffs=False, want_flux=False)
    ctx.set_warm_start(None, True)
    out["coarse start"] = ctx.solve(want_coeffs=False, want_flux=False)
    ctx.set_solver(1e-10, 200, nce.FP64)
    out["coarse start FP64"] = ctx.solve(want_coeffs=False, want_flux=False)
    for name, r in out.items():
        print(f"problem {problem} {name}: {key} {r[key]:.12f}, FP32 {r['iters_fp32']} FP64 {r['iters_fp64']} "
              f"applies, x0 residual {r['rel_residual_x0']:.2e}, fallback {r['used_fallback']}")
        assert r["converged"]
        assert abs(r[key] - out["plain"][key]) < 1e-8 * abs(out["plain"][key])
    assert out["deflated"]["iters_fp32"] < out["plain"]["iters_fp32"]
    assert out["coarse start"]["rel_residual_x0"] < 0.5 and not out["coarse start"]["used_fallback"]
    assert out["coarse start FP64"]["rel_residual_x0"] < 0.5
