"""The per-eps precompute on the GPU (modal solves batched over the
azimuthal orders, Section 9.2; randomized ID on the device, Section 7.1)
against the host precompute: the same one-patch solution and integral vector
to rounding, and system applies that agree to the ID tolerance (the two IDs
draw different sketches and may choose different skeletons, each reproducing
the outgoing field to tol_id). The tree's grids are at 1e-11: the tables'
skeleton sizes enter the tree's cost model, so the two contexts may lay out
different grids, and their interpolation errors must stay below the ID's.
Every other GPU test builds its tables on the GPU as well (the library's
default), so the oracle parity tests cover it."""
import os
import tempfile
import time

import numpy as np
import pytest

import layouts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _ctx(c, eps, problem, host, tol_id, far):
    import paper_1906_04209_amd as nce
    old = os.environ.get("NCE_HOST_PRECOMPUTE")
    os.environ["NCE_HOST_PRECOMPUTE"] = "1" if host else "0"
    try:
        t0 = time.perf_counter()
        ctx = nce.Context(c, eps, problem=problem, tol_id=tol_id, far_field=far, tol_id_fp32=tol_id,
                          tol_grid=1e-11, cache_dir=tempfile.mkdtemp(prefix="nce_tab_"))
        return ctx, time.perf_counter() - t0
    finally:
        if old is None:
            os.environ.pop("NCE_HOST_PRECOMPUTE", None)
        else:
            os.environ["NCE_HOST_PRECOMPUTE"] = old


@pytest.mark.parametrize("problem,eps,N,far", [(1, 0.1, 10, "direct"), (0, 0.01, 1500, "tree")])
def test_gpu_tables_match_host(torch, problem, eps, N, far):
    import paper_1906_04209_amd as nce
    c = layouts.uniform_centers(N, eps, 23)
    ff = nce.FAR_DIRECT if far == "direct" else nce.FAR_TREE
    g, tg = _ctx(c, eps, problem, False, 1e-12, ff)
    h, th = _ctx(c, eps, problem, True, 1e-12, ff)
    Ig, Ih = g.integral_vector(), h.integral_vector()
    eI = np.max(np.abs(Ig - Ih)) / np.max(np.abs(Ih))
    x_np = layouts.random_coeffs(N, g.K, 8, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    yg, yh = g.matvec(x).cpu().numpy(), h.matvec(x).cpu().numpy()
    ey = np.max(np.abs(yg - yh)) / np.max(np.abs(yh - x_np))
    print(f"problem {problem} eps {eps}: tables GPU {tg:.2f} s (p = {g.p}) host {th:.2f} s (p = {h.p}); "
          f"I {eI:.2e}, apply {ey:.2e}")
    assert eI < 1e-13
    assert abs(g.p - h.p) <= max(3, h.p // 20)
    assert ey < 1e-11


def test_gpu_tables_benchmark_eps(torch):
    """The benchmark's tables (interior, eps = 0.001, tol_id 1e-11, with the
    ladder of recompressions): cold build time on the GPU against the host,
    and the ladder's sizes."""
    import paper_1906_04209_amd as nce
    c = layouts.uniform_centers(2000, 0.001, 29)
    g, tg = _ctx(c, 0.001, 0, False, 1e-11, nce.FAR_TREE)
    h, th = _ctx(c, 0.001, 0, True, 1e-11, nce.FAR_TREE)
    x_np = layouts.random_coeffs(len(c), g.K, 9, decay=0.1)
    x = torch.from_numpy(x_np).cuda()
    yg, yh = g.matvec(x).cpu().numpy(), h.matvec(x).cpu().numpy()
    ey = np.max(np.abs(yg - yh)) / np.max(np.abs(yh - x_np))
    print(f"eps 0.001 tables: GPU {tg:.2f} s (p = {g.p}), host {th:.2f} s (p = {h.p}); tree apply difference {ey:.2e}")
    assert ey < 1e-10
