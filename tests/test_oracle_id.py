"""Pin of the oracle's compressed outgoing representation (paper Section 7.1)."""
import math

import numpy as np
import pytest

from oracle import idcomp, onepatch, tables
from oracle.greens import EXTERIOR, INTERIOR, g_surface


def _G(a, b, problem):
    d = np.sqrt(((a[:, None, :] - b[None, :, :]) ** 2).sum(-1))
    return g_surface(d, problem)


@pytest.mark.slow
@pytest.mark.parametrize("problem,eps", [(EXTERIOR, 0.1), (INTERIOR, 0.01)])
def test_skeleton_field_matches_fine_grid(problem, eps):
    # eq. outgoingcompressed: for x in Theta (arclength > 2 eps from the
    # centre), sum_m G(x, s_m) (T f)_m ~ sum_l G(x, x_l^f) (B f)_l w_l
    tol = 1e-12
    res = onepatch.solve_one_patch(eps, problem, M=15)
    cp = idcomp.interpolative_decomposition(res, tol)
    assert 50 < cp.p < 600
    g = np.random.Generator(np.random.PCG64(99))
    n = 300
    r = 2 * eps * np.exp(g.random(n) * np.log(math.pi / (2 * eps) * 0.999))
    r[:60] = 2 * eps * (1 + 1e-6)            # the hardest ring: the boundary of Theta
    th = 2 * math.pi * g.random(n)
    x = idcomp.polar_to_xyz(r, th)
    full = _G(x, idcomp.polar_to_xyz(res.fine_t, res.fine_theta), problem) @ (res.w[:, None] * res.B)
    skel = _G(x, idcomp.polar_to_xyz(cp.skel_t, cp.skel_theta), problem) @ cp.T
    assert np.max(np.abs(full - skel)) <= 10 * tol * np.max(np.abs(full))


@pytest.mark.parametrize("key", ["p0_eps0.1_M15_id1e-12_nt64", "p1_eps0.05_M15_id1e-12_nt64",
                                 "p0_eps0.01_M15_id1e-12_nt64", "p1_eps0.005_M15_id1e-12_nt64",
                                 "p0_eps0.001_M15_id1e-11_nt64"])
def test_outgoing_charges_equal_density_integrals(key):
    # Far from the patch every field is that of its total charge, so the
    # skeleton strengths of basis function k (column k of T, eq.
    # outgoingcompressed) must sum to the integral of its density, I_k of eq.
    # getI, which the oracle gets independently by quadrature of the density
    # profiles. The coarse model's charge chi0 = sum_m T[m][0] rests on this.
    t = tables.load(tables.GOLDEN_DIR / (key + ".npz"))
    err = np.max(np.abs(t.T.sum(axis=0) - t.I)) / np.max(np.abs(t.I))
    print(f"{key}: p = {t.p}, max |sum_m T[m][k] - I_k| / max |I| = {err:.2e}")
    assert err < 1e-10
