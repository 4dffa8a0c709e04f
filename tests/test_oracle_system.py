"""Pins of the oracle's many-patch system, solver and scalars (paper Sections 2, 3, 6, 8)."""
import math

import numpy as np
import pytest

import layouts
from oracle import csum, greens, onepatch, system, tables
from oracle.greens import EXTERIOR, INTERIOR


@pytest.fixture(scope="module")
def tab_e():
    return tables.get(EXTERIOR, 0.1, 15, 1e-12)


@pytest.fixture(scope="module")
def tab_i():
    return tables.get(INTERIOR, 0.1, 15, 1e-12)


_FULL = {}


def _full(problem):
    """(Tables, OnePatch) at eps = 0.1, computed once per module."""
    if problem not in _FULL:
        from conftest import oracle_onepatch
        _FULL[problem] = oracle_onepatch(problem, 0.1)
    return _FULL[problem]


def test_single_patch(tab_i, tab_e):
    # N = 1: the system is the identity, x = e_0, I_sigma = I_0, mu = 1/(3 I_0) - 3/5
    for tab in (tab_i, tab_e):
        lay = system.Layout(np.array([[0.0, 0.6, 0.8]]), tab)
        r = system.solve_gmres(lay, tol=1e-14)
        assert r["iters"] == 0 or np.allclose(r["x"], system.rhs(1, tab.K), atol=1e-15)
        assert abs(r["I_sigma"] - tab.I[0]) < 1e-16
    r = system.solve_dense(system.Layout(np.array([[1.0, 0, 0]]), tab_i))
    assert abs(r["mu"] - (1 / (3 * tab_i.I[0]) - 0.6)) < 1e-14


def test_dense_lu_equals_gmres(tab_e):
    c = layouts.uniform_centers(10, 0.1, 1)
    lay = system.Layout(c, tab_e)
    a = system.solve_dense(lay)
    b = system.solve_gmres(lay, tol=1e-13)
    assert abs(a["capture_rate"] - b["capture_rate"]) < 1e-12 * a["capture_rate"]
    assert np.max(np.abs(a["x"] - b["x"])) < 1e-11
    assert 4 <= b["iters"] <= 14


def test_antipodal_pair_symmetry(tab_i):
    c = np.array([[0.0, 0.0, 1.0], [0.0, 0.0, -1.0]])
    r = system.solve_dense(system.Layout(c, tab_i))
    assert abs(r["flux"][0] - r["flux"][1]) < 1e-15
    assert np.max(np.abs(np.abs(r["x"][0]) - np.abs(r["x"][1]))) < 1e-14


def test_rotation_permutation_invariance(tab_e):
    c = layouts.uniform_centers(8, 0.1, 21)
    base = system.solve_dense(system.Layout(c, tab_e))
    g = np.random.Generator(np.random.PCG64(4))
    Qm, _ = np.linalg.qr(g.standard_normal((3, 3)))
    perm = g.permutation(8)
    c2 = (c @ Qm.T)[perm]
    other = system.solve_dense(system.Layout(c2, tab_e))
    assert abs(other["capture_rate"] - base["capture_rate"]) < 1e-12 * base["capture_rate"]
    assert np.max(np.abs(other["flux"] - base["flux"][perm])) < 1e-13


def test_scalar_bounds(tab_i, tab_e):
    # full coverage gives mu = 1/15 (mean G_I = 2 => I_sigma = 1/2) and capture
    # rate 4 pi (mean G_E = 1 => I_sigma = 1); partial coverage lies beyond those bounds.
    c = layouts.uniform_centers(12, 0.1, 8)
    ri = system.solve_dense(system.Layout(c, tab_i))
    re = system.solve_dense(system.Layout(c, tab_e))
    assert ri["mu"] > 1 / 15
    assert 0 < re["capture_rate"] < 4 * math.pi
    # the paper's J is minus I_sigma; the capture rate is 4 pi I_sigma
    assert abs(re["J_paper"] + re["I_sigma"]) == 0.0


@pytest.mark.slow
def test_compressed_equals_uncompressed():
    # the ID (Section 7.1) changes the system only at the level of tol_id
    tab, res = _full(EXTERIOR)
    c = layouts.uniform_centers(4, 0.1, 31)
    lay = system.Layout(c, tab)
    x = layouts.random_coeffs(4, tab.K, 5, decay=0.2)
    yc = system.matvec_dense(lay, x)
    yu = system.matvec_uncompressed(lay, res, x)
    assert np.max(np.abs(yc - yu)) < 1e-10 * np.max(np.abs(yu - x))
    bu = np.linalg.solve
    # solutions: compressed dense LU vs GMRES on the uncompressed operator
    rc = system.solve_dense(lay)
    xu, it, _ = system.gmres(lambda v: system.matvec_uncompressed(lay, res, v),
                             system.rhs(4, tab.K), 1e-13)
    Iu = float(np.sum(xu @ tab.I))
    assert abs(Iu - rc["I_sigma"]) < 1e-10 * rc["I_sigma"]


@pytest.mark.slow
def test_fibonacci_table2_plausibility():
    # Table 2 (Fibonacci spiral, f = 0.05, N = 10, interior, M = 15) prints
    # mu = 0.62771752. The spiral variant the paper cites is not given, so the
    # published digits cannot be reproduced exactly. The "ends" variant
    # (z_k = 1 - 2k/(N-1), golden-angle azimuth) lands within 0.2 % of the
    # printed value; the "half" variant (z_k = 1 - (2k+1)/N) lands 1.8 % off,
    # so only "ends" serves as the pin. A sign or scaling error in the kernel
    # or in the mu formula moves mu by tens of percent (the printed modal
    # signs give 0.43).
    N = 10
    eps = layouts.eps_from_area_fraction(0.05, N)
    tab = tables.get(INTERIOR, eps, 15, 1e-12)
    c = layouts.fibonacci_centers(N, "ends")
    r = system.solve_dense(system.Layout(c, tab))
    assert abs(r["mu"] - 0.62771752) < 0.002 * 0.62771752, r["mu"]


@pytest.mark.slow
@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_csum_matches_dense_incoming(problem):
    """The oracle's C all-pairs loop (csum.c), which writes the stored matvec
    rows the GPU is compared with, against the plain numpy sum
    system.incoming_dense (eq. sysmatapply's scattered field, both Green's
    functions of Section 2.1). Independent code paths: a swapped problem flag,
    a dropped self-exclusion or an index slip in either shows here."""
    tab = tables.get(problem, 0.1, 15, 1e-12)
    for N, seed, targets in ((10, 1, None), (40, 61, [0, 17, 39])):
        lay = system.Layout(layouts.uniform_centers(N, 0.1, seed), tab)
        x = layouts.random_coeffs(N, tab.K, 900 + N, decay=0.1)
        ref = system.incoming_dense(lay, x, targets)
        got = csum.incoming_layout(lay, x, targets)
        assert got.shape == ref.shape
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)), np.max(np.abs(got - ref))
    # the problem flag matters: the other problem's kernel gives a different field
    other = csum.incoming(1 - problem, lay.Z, lay.S, x @ tab.T.T, [0])
    assert np.max(np.abs(other - ref[:1])) > 1e-3 * np.max(np.abs(ref))


@pytest.mark.slow
def test_capture_rate_flat_disk_limit():
    """Capture rate normalisation 4 pi I_sigma (the flux magnitude of eq. flux,
    Section 2.2) through scalars(): one exterior patch of radius eps becomes a
    flat disk as eps -> 0, whose capture rate on a reflecting plane is 4 eps
    (the Weber disk's one-sided flux; Berg and Purcell). The relative gap
    rate / (4 eps) - 1 shrinks like (eps / pi) log(2 / eps), the size of the
    log(2/d) term of G_E over the patch. A 2 pi (or 1) normalisation would put
    the ratio near 1/2 (or 1 / 4 pi)."""
    prev = math.inf
    for eps in (0.1, 0.03, 0.01, 0.003):
        op = onepatch.solve_one_patch(eps, EXTERIOR, M=0)
        tab = system.Tables(EXTERIOR, eps, 0, np.zeros((1, 1)), np.zeros(1), np.zeros(1), op.I,
                            np.ones((1, 1)), np.zeros(1), np.zeros(1))
        r = system.scalars(tab, system.rhs(1, 1))   # N = 1: x = e_0
        gap = r["capture_rate"] / (4 * eps) - 1
        lead = eps / math.pi * math.log(2 / eps)
        assert 0 < gap < prev
        assert 0.9 * lead < gap < 1.25 * lead, (eps, gap, lead)
        prev = gap
    assert abs(gap / lead - 1) < 0.05


@pytest.mark.slow
def test_interior_flux_identity():
    """Divergence theorem for the interior problem (Section 2.3): v = sum_i
    S_i[sigma_i] has the same normal derivative, -I_sigma, at every point of
    the reflecting surface (Lemma intsigma), so vbar = (v - 1) / (3 D) +
    (1 - |x|^2) / 6 with D = -I_sigma has zero flux there and the whole escape
    flux through the patches is the ball's volume 4 pi / 3. The derivative is
    taken numerically from the off-surface Green's function on interior points
    and compared with I_sigma from the integral vector I. This holds for any
    densities (it checks G_I's Neumann property and I as the integral of
    sigma); that the densities solve the system is checked on the patches by
    test_dirichlet_condition_on_patches."""
    tab, res = _full(INTERIOR)
    c = layouts.uniform_centers(4, 0.1, 41)
    lay = system.Layout(c, tab)
    r = system.solve_dense(lay)
    Is = r["I_sigma"]
    Xf = system.patch_points(lay.c, lay.e1, lay.e2, res.fine_t, res.fine_theta)   # (N, n_f, 3)
    sw = (r["x"] @ res.B.T) * res.w[None, :]                                      # sigma_j dS

    def v(y):
        return sum(float(np.sum(greens.g_offsurface(y[None, :], Xf[j], INTERIOR) * sw[j])) for j in range(lay.N))

    g = np.random.default_rng(7)
    checked = 0
    while checked < 6:
        x = g.standard_normal(3)
        x /= np.linalg.norm(x)
        if np.min(np.arccos(np.clip(lay.c @ x, -1, 1))) < 0.4:   # stay clear of the patches (eps = 0.1)
            continue
        h = 1e-5
        # one-sided second-order difference along the outward normal
        dvdn = (3 * v(x) - 4 * v((1 - h) * x) + v((1 - 2 * h) * x)) / (2 * h)
        assert abs(dvdn + Is) < 1e-7 * abs(Is), (dvdn, -Is)
        checked += 1
    # with D = -I_sigma the flux of vbar through the patches: (1/(3D)) * (-D |Gamma_R|) - |Gamma_A|/3 = -4 pi/3
    area_a = lay.N * 2 * math.pi * (1 - math.cos(0.1))
    D = -Is
    flux_a = (1.0 / (3.0 * D)) * (-D * (4 * math.pi - area_a)) - area_a / 3.0
    assert abs(flux_a + 4 * math.pi / 3) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_dirichlet_condition_on_patches(problem):
    """v = 1 on every patch (the absorbing condition, Sections 2.2 and 2.3) at
    random points off the discretization grids, for the solved densities; a
    relative change of 1e-6 in one patch's leading coefficient breaks it by
    that much."""
    tab, res = _full(problem)
    eps = 0.1
    for N, seed in ((4, 41), (8, 42)):
        lay = system.Layout(layouts.uniform_centers(N, eps, seed), tab)
        x = system.solve_dense(lay)["x"]
        g = np.random.default_rng(3)
        for i in range(N):
            t = eps * np.sqrt(g.random(30))
            th = 2 * np.pi * g.random(30)
            assert np.max(np.abs(system.patch_residual(lay, res, x, i, t, th))) < 1e-11
        xp = x.copy()
        xp[0, 0] *= 1 + 1e-6
        assert np.max(np.abs(system.patch_residual(lay, res, xp, 0, t, th))) > 5e-7

