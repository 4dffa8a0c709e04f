"""Benchmark: GMRES matrix-vector products per second of the narrow capture /
narrow escape system, plus time to a 1e-8 relative residual, on one MI355X.

One step = one application of the FP64 system matrix (Section 8, Step 3,
items 1-5) to a seeded random coefficient vector. Inputs are resident in HBM
before the timed region. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg5]
                  [--precision fp64|mixed] [--no-solve] [--no-warm] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import layouts  # noqa: E402

# Green's function pair cost in lane-cycles: the VALU instructions of the P2L
# inner loop (AMD assembly of this build, 4 pairs per iteration) priced at the
# chip's issue rates -- FP64 add/mul/fma and 64-bit integer ops 1 (78.6 TFLOP/s
# FP64 vector), 32-bit ops 0.5 (157.3 TFLOP/s FP32 vector), FP32
# transcendentals 2, FP64 rcp/rsq 4. The ALU ceiling is
# 256 CUs * 64 lanes * 2.4 GHz / c_pair pairs per second.
C_PAIR = {("fp64", 0): 68.1, ("fp64", 1): 55.1, ("fp32", 0): 12.4, ("fp32", 1): 9.4}
LANE_CYCLES_PER_S = 256 * 64 * 2.4e9
WARM_WEIGHTS = __import__("pathlib").Path(ROOT) / "paper_1906_04209_amd" / "weights" / "warmstart.npz"

WORKLOADS = {
    "cfg5": dict(layouts.CONFIGS["cfg5"], far="tree"),
    "cfg2": dict(layouts.CONFIGS["cfg2"], far="direct"),
    "cfg3": dict(layouts.CONFIGS["cfg3"], far="tree"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, tol_id, x, centers, nrows=1):
    """Time the oracle's dense compressed matvec on `nrows` sampled target
    patches (plain C loop over all N source patches, all host cores) and scale
    to one full matvec."""
    from oracle import csum, system, tables
    tab = tables.get(cfg["problem"], cfg["eps"], 15, tol_id)
    lay = system.Layout(centers, tab)
    rows = np.arange(nrows)
    t0 = time.perf_counter()
    U = csum.incoming_layout(lay, x, rows)
    y = x[rows] + U @ tab.P.T
    dt = time.perf_counter() - t0
    per_matvec = dt * cfg["N"] / nrows
    cores = len(os.sched_getaffinity(0))
    return {"value": 1.0 / per_matvec, "unit": "matvec/s", "cores": cores, "kind": "oracle",
            "sample": f"{nrows} of {cfg['N']} target patches of the dense compressed matvec "
                      f"({dt:.1f} s), scaled by N/{nrows}",
            "seconds_per_matvec_extrapolated": per_matvec}, rows, y


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-solve", action="store_true", help="skip the FP64 and mixed solves to 1e-8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-warm", action="store_true", help="skip the solves from the learned initial guess")
    ap.add_argument("--tol-id", type=float, default=1e-11)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); nothing in this build uses a second GPU.",
              file=sys.stderr)
        sys.exit(2)

    os.environ.setdefault("NCE_CACHE", "/tmp")
    import torch
    import paper_1906_04209_amd as nce

    cfg = WORKLOADS[args.workload]
    t0 = time.time()
    centers = layouts.config_layout(cfg)
    log(f"layout {args.workload}: N={cfg['N']} eps={cfg['eps']} ({time.time() - t0:.1f} s)")
    far = nce.FAR_TREE if cfg["far"] == "tree" else nce.FAR_DIRECT
    prec = nce.FP64 if args.precision == "fp64" else nce.MIXED
    t0 = time.time()
    ctx = nce.Context(centers, cfg["eps"], problem=cfg["problem"], tol_id=args.tol_id, far_field=far)
    t_setup = time.time() - t0
    work = ctx.work()
    log(f"setup {t_setup:.1f} s: K={ctx.K} K*={ctx.Kstar} p={ctx.p} levels={ctx.levels} work={work}")
    x_np = layouts.random_coeffs(cfg["N"], ctx.K, 777, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    y = ctx.empty()
    torch.cuda.synchronize()
    for w in range(args.warmup):
        ctx.matvec_profile(x, y, prec)
        log(f"warmup {w + 1}/{args.warmup}")
    torch.cuda.synchronize()
    steps_ms = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        _, ms = ctx.matvec_profile(x, y, prec)
        steps_ms.append(ms)
        log(f"step {k + 1}/{args.steps}: {ms.sum():.2f} ms {np.round(ms, 3).tolist()}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    st = np.mean(np.array(steps_ms), axis=0)
    dom = 1  # far field (direct all-pairs sum or P2L)
    pairs = work["pairs_far"]
    ptag = "fp64" if prec == nce.FP64 else "fp32"
    cp = C_PAIR[(ptag, cfg["problem"])]
    achieved = pairs / (st[dom] * 1e-3)
    peak = LANE_CYCLES_PER_S / cp
    out = {
        "metric": "GMRES matvecs/s (FP64 system apply) at N=1e5; time to 1e-8 residual reported alongside",
        "value": 1e3 / ms_step, "unit": "matvec/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == nce.FP64 else "f32+f64", "data": "synthetic",
        "config": {"workload": args.workload, "N": cfg["N"], "eps": cfg["eps"],
                   "problem": "interior" if cfg["problem"] == 0 else "exterior", "far_field": cfg["far"],
                   "K": ctx.K, "Kstar": ctx.Kstar, "p": ctx.p, "levels": ctx.levels, "tol_id": args.tol_id,
                   "layout": cfg["layout"], "seed": cfg["seed"]},
        "step_ms": {"block_apply": st[0], "far": st[1], "near": st[2], "interp": st[3], "p_apply": st[4]},
        "setup_s": t_setup,
        "roofline": {"bound": "alu", "kernel": "far-field Green's sum", "achieved": achieved / 1e9,
                     "peak": peak / 1e9, "unit": "Gpair/s", "frac": achieved / peak, "traffic": None,
                     "c_pair_lane_cycles": cp, "pairs_per_launch": pairs},
    }
    if not args.no_solve:
        # time to a 1e-8 relative residual (FP64-verified), from x0 = 0
        for name, pr in (("fp64", nce.FP64), ("mixed", nce.MIXED)):
            ctx.set_solver(1e-8, 100, pr)
            r = ctx.solve(want_coeffs=False, want_flux=False)
            key = "mu" if cfg["problem"] == 0 else "capture_rate"
            out[f"solve_{name}"] = {k: r[k] for k in ("iters_fp64", "iters_fp32", "outer", "rel_residual",
                                                       "t_solve_s", "converged")}
            out[f"solve_{name}"][key] = r[key]
            log(f"solve {name}: {out[f'solve_{name}']}")
        a, b = out["solve_fp64"], out["solve_mixed"]
        key = "mu" if cfg["problem"] == 0 else "capture_rate"
        out["time_to_1e-8_s"] = {"fp64": a["t_solve_s"], "mixed": b["t_solve_s"],
                                 "speedup": a["t_solve_s"] / b["t_solve_s"],
                                 f"rel_diff_{key}": abs(a[key] - b[key]) / abs(a[key])}
        if not args.no_warm and WARM_WEIGHTS.exists():
            # the same solves from the learned initial guess (the first one also
            # computes the per-patch features, which is counted in its time)
            from paper_1906_04209_amd import warmstart
            net = warmstart.load(WARM_WEIGHTS)
            ctx.set_warm_start(net)
            for name, pr in (("fp64", nce.FP64), ("mixed", nce.MIXED)):
                ctx.set_solver(1e-8, 100, pr)
                r = ctx.solve(want_coeffs=False, want_flux=False)
                o = {k: r[k] for k in ("iters_fp64", "iters_fp32", "outer", "rel_residual", "rel_residual_x0",
                                       "used_fallback", "t_solve_s", "converged")}
                o[key] = r[key]
                o[f"rel_diff_{key}_vs_cold"] = abs(r[key] - a[key]) / abs(a[key])
                out[f"solve_{name}_warm"] = o
                out["time_to_1e-8_s"][f"{name}_warm"] = r["t_solve_s"]
                log(f"solve {name} warm: {o}")
            ctx.set_warm_start(None)
    if not args.no_cpu_baseline:
        cb, rows, yref = cpu_baseline(cfg, args.tol_id, x_np, centers)
        yg = y.cpu().numpy()[rows] if args.precision == "fp64" else None
        if yg is not None:
            cb["parity_rel_err_sampled_rows"] = float(np.max(np.abs(yg - yref)) / np.max(np.abs(yref - x_np[rows])))
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
