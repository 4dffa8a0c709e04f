"""GPU checks of the coarse-space deflation of the mixed solves: its coarse
matrix against the same quantity formed from the oracle's closed-form Green's
function, and mixed solves with and without it (same result, fewer FP32
applies)."""
import numpy as np
import pytest

import layouts
from test_host_deflate import harmonic_polys, mgs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("prob,N,eps,seed", [(0, 300, 0.02, 3), (1, 700, 0.01, 4)])
def test_deflation_matrix_matches_closed_form(torch, prob, N, eps, seed):
    import paper_1906_04209_amd as nce
    from oracle import greens
    c = layouts.uniform_centers(N, eps, seed)
    ctx = nce.Context(c, eps, problem=prob, tol_id=1e-11)
    _, _, chi0 = ctx.coarse(with_chi0=True)
    k, T = ctx.deflation_matrix()
    assert k == 16
    Z = mgs(harmonic_polys(c))
    d = np.linalg.norm(c[:, None, :] - c[None, :, :], axis=-1)
    np.fill_diagonal(d, 1.0)
    G = greens.g_surface(d, prob)
    np.fill_diagonal(G, 0.0)
    ref = np.eye(16) + chi0 * (Z.T @ G @ Z)
    err = np.max(np.abs(T - ref)) / np.max(np.abs(ref - np.eye(16)))
    print(f"problem {prob} N={N}: deflation matrix rel err {err:.2e}, diagonal {np.diag(ref)[:4]}")
    assert err < 1e-5


def test_deflation_keeps_result_and_saves_applies(torch):
    import paper_1906_04209_amd as nce
    c = layouts.uniform_centers(3000, 0.005, 77)
    out = {}
    for defl in (False, True):
        ctx = nce.Context(c, 0.005, problem=nce.INTERIOR, tol_id=1e-11, tol_gmres=1e-10, precision=nce.MIXED,
                          deflation=defl)
        r = ctx.solve(want_coeffs=False, want_flux=False)
        assert r["converged"]
        out[defl] = r
        print(f"deflation {defl}: FP32 applies {r['iters_fp32']}, FP64 {r['iters_fp64']}, mu {r['mu']:.12f}, "
              f"residual {r['rel_residual']:.2e}")
    rel = abs(out[True]["mu"] - out[False]["mu"]) / out[False]["mu"]
    assert rel < 1e-8
    assert out[True]["iters_fp32"] < out[False]["iters_fp32"]
