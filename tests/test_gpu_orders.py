"""Basis orders other than the paper's M = 15 (K = (M+1)(M+2)/2 Zernike
functions, K* = (M+1)(2M+2) sampling nodes): the all-pairs apply and solve
against the oracle's stored values (tests/golden/orders_*.npz, written by
make_golden.py), and the tree apply, whose interpolation kernel applies P
through its factors with rings of 2M+2 nodes (zero padded when 2M+2 is not a
multiple of the 16-byte read), against the all-pairs apply."""
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


@pytest.mark.parametrize("M,problem", [(4, 1), (10, 0)])
def test_orders_vs_oracle(torch, M, problem):
    import paper_1906_04209_amd as nce
    g = np.load(GOLD / f"orders_M{M}_p{problem}.npz")
    cfg = layouts.CONFIGS["cfg1"]
    c = layouts.config_layout(cfg)
    ctx = nce.Context(c, cfg["eps"], problem=problem, M=M, tol_id=1e-12, far_field=nce.FAR_DIRECT,
                      tol_gmres=1e-12)
    assert ctx.K == (M + 1) * (M + 2) // 2 and ctx.Kstar == (M + 1) * (2 * M + 2)
    x = layouts.random_coeffs(cfg["N"], ctx.K, int(g["x_seed"]), decay=0.1)
    xd = torch.from_numpy(x).cuda()
    ref = g["y"]
    err = np.max(np.abs(ctx.matvec(xd).cpu().numpy() - ref)) / np.max(np.abs(ref - x))
    errm = np.max(np.abs(ctx.matvec(xd, precision=nce.MIXED).cpu().numpy() - ref)) / np.max(np.abs(ref - x))
    r = ctx.solve(want_coeffs=False)
    key = "capture_rate" if problem == 1 else "mu"
    rel = abs(r[key] - float(g["scalar"])) / abs(float(g["scalar"]))
    flux_err = np.max(np.abs(r["flux"].cpu().numpy() - g["flux"])) / np.max(np.abs(g["flux"]))
    print(f"M={M} problem {problem}: matvec FP64 {err:.2e} FP32 {errm:.2e}; {key} {r[key]:.15f} vs "
          f"{float(g['scalar']):.15f} rel {rel:.2e}; flux {flux_err:.2e}")
    assert err < 1e-12 and errm < 2e-5
    assert rel < 1e-11 and flux_err < 1e-10


@pytest.mark.parametrize("M", [6, 14])
def test_tree_fused_p_apply_other_orders(torch, M):
    import paper_1906_04209_amd as nce
    N, eps = 2000, 0.005
    c = layouts.uniform_centers(N, eps, 21)
    d = nce.Context(c, eps, problem=0, M=M, tol_id=1e-12, far_field=nce.FAR_DIRECT)
    t = nce.Context(c, eps, problem=0, M=M, tol_id=1e-12, tol_grid=1e-8, far_field=nce.FAR_TREE,
                    tol_grid_fp32=1e-4, tol_id_fp32=1e-6)
    x_np = layouts.random_coeffs(N, d.K, 9, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    yd = d.matvec(x).cpu().numpy()
    scale = np.max(np.abs(yd - x_np))
    err = np.max(np.abs(t.matvec(x).cpu().numpy() - yd)) / scale
    errm = np.max(np.abs(t.matvec(x, precision=nce.MIXED).cpu().numpy() - yd)) / scale
    print(f"M={M} (K={t.K}, K*={t.Kstar}), levels {t.levels}: tree vs direct FP64 {err:.2e}, FP32 {errm:.2e}")
    assert err < 3e-9
    assert errm < 2e-5
