"""Write the oracle's stored expected values used by the GPU parity tests.

Calls only `oracle/` and the seeded generators in `layouts`. Outputs (under
tests/golden/):
  tables/<key>.npz      oracle precompute (T, skeleton, I) per (problem, eps, M, tol_id)
  cfg1.npz              N=10 exterior, eps=0.1, seed 1: matvec of seeded x, dense-LU solve
  cfg1i.npz             the same centres, interior: matvec of seeded x, dense-LU solve (mu,
                        I_sigma, per-patch flux, solution coefficients)
  mt_p<problem>.npz     N=10 with two patch radii (0.1 and 0.05, seed 51), both problems: matvec of
                        seeded x, the dense-LU solve (scalars, per-patch flux, coefficients), and the
                        solution's field at seeded points and eq. l2res on a patch of each radius
  orders_M<M>_p<problem>.npz  the cfg1 centres at basis orders other than 15 (M = 4 exterior, M = 10
                        interior): matvec of seeded x and the dense-LU scalars
  cfg2_rows.npz         N=1000 interior, eps=0.01, seed 2: matvec rows at 16 sampled patches
  cfg3_rows.npz         N=10000 exterior clustered, eps=0.005, seed 3: 12 sampled rows
  cfg5_rows.npz         N=100000 interior, eps=0.001, seed 5: 16 sampled rows (tol_id 1e-11)
  MANIFEST.json         SHA-256 of every file, with the command that made it

Run:  python tests/golden/make_golden.py [name ...]
"""
from __future__ import annotations

import hashlib
import json
import sys
import time
from pathlib import Path

import numpy as np

ROOT = Path(__file__).resolve().parents[2]
sys.path.insert(0, str(ROOT))

import layouts  # noqa: E402
from oracle import csum, multitype, system, tables  # noqa: E402

GOLD = ROOT / "tests" / "golden"
TOL_ID = 1e-12
X_SEED = 777          # seed of the matvec input vectors
ROW_SEED = 4242       # seed of the sampled target patches


def _tab(problem, eps):
    k = tables.key(problem, eps, 15, TOL_ID)
    f = tables.GOLDEN_DIR / (k + ".npz")
    if f.exists():
        return tables.load(f)
    t0 = time.time()
    tab, _, _ = tables.compute(problem, eps, 15, TOL_ID)
    tables.save(tab, f)
    print(f"  tables {k}: p={tab.p} ({time.time() - t0:.0f} s)", flush=True)
    return tab


def make_cfg1():
    cfg = layouts.CONFIGS["cfg1"]
    tab = _tab(cfg["problem"], cfg["eps"])
    c = layouts.config_layout(cfg)
    lay = system.Layout(c, tab)
    x = layouts.random_coeffs(cfg["N"], tab.K, X_SEED, decay=0.1)
    y = system.matvec_dense(lay, x)
    r = system.solve_dense(lay)
    it = system.solve_gmres(lay, tol=1e-10)
    np.savez(GOLD / "cfg1.npz", y=y, x_seed=X_SEED, capture_rate=r["capture_rate"], I_sigma=r["I_sigma"],
             flux=r["flux"], gmres_iters=it["iters"])
    print(f"  cfg1 capture rate {r['capture_rate']:.15g}, GMRES iters {it['iters']}", flush=True)


def make_cfg1i():
    """Interior twin of cfg1 (same centres): the narrow escape scalars of
    Section 2.3 (eq. mufromsigma2) and the per-patch flux from the dense LU
    solve of the compressed system."""
    cfg = layouts.CONFIGS["cfg1"]
    tab = _tab(0, cfg["eps"])
    c = layouts.config_layout(cfg)
    lay = system.Layout(c, tab)
    x = layouts.random_coeffs(cfg["N"], tab.K, X_SEED, decay=0.1)
    y = system.matvec_dense(lay, x)
    r = system.solve_dense(lay)
    it = system.solve_gmres(lay, tol=1e-10)
    np.savez(GOLD / "cfg1i.npz", y=y, x_seed=X_SEED, mu=r["mu"], I_sigma=r["I_sigma"], flux=r["flux"],
             coeffs=r["x"], gmres_iters=it["iters"])
    print(f"  cfg1i mu {r['mu']:.15g}, GMRES iters {it['iters']}", flush=True)


MT_RADII = (0.1, 0.05)
MT_SEED = 51


def _mt_field_points(lay, problem, seed):
    """Targets of the two-radius field check: eps_j/5 off patches of both
    radii, on them, on the reflecting surface, near it and deep in the domain."""
    g = np.random.default_rng(seed)
    sgn = -1.0 if problem == 0 else 1.0
    pts = []
    for i in (int(np.flatnonzero(lay.types == 0)[0]), int(np.flatnonzero(lay.types == 1)[0])):
        eps = lay.tab(i).eps
        t = eps * np.sqrt(g.random(3))
        th = 2 * np.pi * g.random(3)
        on = system.patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], t, th)[0]
        pts += [(1.0 + sgn * eps / 5) * on[0], (1.0 + sgn * eps / 5) * on[1], on[2]]
    while len(pts) < 9:
        d = g.standard_normal(3)
        d /= np.linalg.norm(d)
        if np.min(np.arccos(np.clip(lay.c @ d, -1, 1))) > 0.3:
            pts += [d, (1.0 + sgn * 1e-3) * d]
    pts += [np.array([0.1, -0.2, 0.3]) if problem == 0 else np.array([1.5, -0.4, 0.9])]
    return np.array(pts)


def make_mt():
    """Two patch radii in one configuration (oracle/multitype.py): apply,
    dense solve, and the field of the solution (potential at seeded points,
    eq. l2res on one patch of each radius)."""
    c, types = layouts.multi_radius_centers(10, MT_RADII, MT_SEED)
    for problem in (0, 1):
        tabs = [_tab(problem, e) for e in MT_RADII]
        ops = [tables.compute(problem, e, 15, TOL_ID)[1] for e in MT_RADII]
        lay = multitype.Layout(c, types, tabs)
        x = layouts.random_coeffs(10, tabs[0].K, X_SEED, decay=0.1)
        y = multitype.matvec_dense(lay, x)
        r = multitype.solve_dense(lay)
        extra = {"mu": r["mu"]} if problem == 0 else {"capture_rate": r["capture_rate"]}
        fpts = _mt_field_points(lay, problem, 90 + problem)
        fval = multitype.potential(lay, ops, r["x"], fpts)
        rpat = np.array([int(np.flatnonzero(types == 0)[0]), int(np.flatnonzero(types == 1)[0])])
        rval = np.array([multitype.l2_residual(lay, ops, r["x"], int(i), nt=6, ntheta=10)[0] for i in rpat])
        np.savez(GOLD / f"mt_p{problem}.npz", y=y, x_seed=X_SEED, I_sigma=r["I_sigma"], flux=r["flux"],
                 coeffs=r["x"], types=types, radii=np.array(MT_RADII), seed=MT_SEED, field_points=fpts,
                 field_values=fval, residual_patches=rpat, residual_values=rval, **extra)
        print(f"  mt problem {problem}: types {types.tolist()} I_sigma {r['I_sigma']:.15g}; "
              f"residuals {rval}", flush=True)


def make_cfg2_rows():
    cfg = layouts.CONFIGS["cfg2"]
    tab = _tab(cfg["problem"], cfg["eps"])
    c = layouts.config_layout(cfg)
    lay = system.Layout(c, tab)
    x = layouts.random_coeffs(cfg["N"], tab.K, X_SEED, decay=0.1)
    rows = np.sort(layouts.rng(ROW_SEED).choice(cfg["N"], 16, replace=False))
    U = csum.incoming_layout(lay, x, rows)
    y = x[rows] + U @ tab.P.T
    np.savez(GOLD / "cfg2_rows.npz", rows=rows, y=y, x_seed=X_SEED)
    print(f"  cfg2 rows {rows.tolist()}", flush=True)


def _rows_job(name, nrows, tol_id):
    def job():
        cfg = layouts.CONFIGS[name]
        k = tables.key(cfg["problem"], cfg["eps"], 15, tol_id)
        f = tables.GOLDEN_DIR / (k + ".npz")
        if f.exists():
            tab = tables.load(f)
        else:
            tab, _, _ = tables.compute(cfg["problem"], cfg["eps"], 15, tol_id)
            tables.save(tab, f)
        c = layouts.config_layout(cfg)
        lay = system.Layout(c, tab)
        x = layouts.random_coeffs(cfg["N"], tab.K, X_SEED, decay=0.1)
        rows = np.sort(layouts.rng(ROW_SEED).choice(cfg["N"], nrows, replace=False))
        t0 = time.time()
        U = csum.incoming_layout(lay, x, rows)
        y = x[rows] + U @ tab.P.T
        np.savez(GOLD / f"{name}_rows.npz", rows=rows, y=y, x_seed=X_SEED, tol_id=tol_id)
        print(f"  {name} rows {rows.tolist()} ({time.time() - t0:.0f} s)", flush=True)
    return job


def make_orders():
    """Basis orders other than the paper's M = 15 (its P, nodes and skeletons
    all change with M)."""
    cfg = layouts.CONFIGS["cfg1"]
    c = layouts.config_layout(cfg)
    for problem, M in ((1, 4), (0, 10)):
        t0 = time.time()
        tab, _, _ = tables.compute(problem, cfg["eps"], M, TOL_ID)
        lay = system.Layout(c, tab)
        x = layouts.random_coeffs(cfg["N"], tab.K, X_SEED, decay=0.1)
        y = system.matvec_dense(lay, x)
        r = system.solve_dense(lay)
        key = "capture_rate" if problem == 1 else "mu"
        np.savez(GOLD / f"orders_M{M}_p{problem}.npz", y=y, x_seed=X_SEED, M=M, problem=problem,
                 eps=cfg["eps"], scalar=r[key], flux=r["flux"])
        print(f"  orders M={M} problem {problem}: {key} {r[key]:.15g} ({time.time() - t0:.0f} s)", flush=True)


JOBS = {"cfg1": make_cfg1, "cfg1i": make_cfg1i, "mt": make_mt, "orders": make_orders, "cfg2_rows": make_cfg2_rows,
        "cfg3_rows": _rows_job("cfg3", 12, 1e-12), "cfg5_rows": _rows_job("cfg5", 16, 1e-11)}


def manifest():
    out = {"command": "python tests/golden/make_golden.py", "files": {}}
    for f in sorted(GOLD.rglob("*.npz")):
        out["files"][str(f.relative_to(GOLD))] = hashlib.sha256(f.read_bytes()).hexdigest()
    (GOLD / "MANIFEST.json").write_text(json.dumps(out, indent=1) + "\n")


if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    for n in names:
        print(n, flush=True)
        JOBS[n]()
    manifest()
