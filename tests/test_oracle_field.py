"""Pins of the oracle's field evaluation (oracle/field.py; paper Sections 2.1-2.3
and eq. l2res): properties the Neumann Green's functions and the
representation fix exactly, checked on solved layouts of a few patches."""
import math

import numpy as np
import pytest

import layouts
from oracle import field, system, tables
from oracle.greens import EXTERIOR, INTERIOR

pytestmark = pytest.mark.slow
EPS = 0.1
_CACHE = {}


def _solved(problem):
    if problem not in _CACHE:
        from conftest import oracle_onepatch
        tab, op = oracle_onepatch(problem, EPS)
        lay = system.Layout(layouts.uniform_centers(5, EPS, 71), tab)
        x = system.solve_dense(lay)["x"]
        _CACHE[problem] = (lay, op, x)
    return _CACHE[problem]


def _reflecting_points(lay, n, seed, clearance=0.4):
    g = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        p = g.standard_normal(3)
        p /= np.linalg.norm(p)
        if np.min(np.arccos(np.clip(lay.c @ p, -1, 1))) > clearance:
            out.append(p)
    return np.array(out)


def test_interior_value_at_centre():
    # G_I(0, x') = 2 for x' on the sphere (eq. Gintoffsurface), so v(0) = 2 I_sigma
    lay, op, x = _solved(INTERIOR)
    Is = float(np.sum(x @ lay.tab.I))
    v0 = field.potential(lay, op, x, np.zeros((1, 3)))[0]
    assert abs(v0 - 2 * Is) < 1e-13 * abs(Is), (v0, 2 * Is)


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_normal_derivative_on_reflecting_surface(problem):
    # interior: dv/dn = -I_sigma (Lemma intsigma); exterior: du/dn = 0 (G_E's
    # Neumann condition); one-sided second-order differences from the domain side
    lay, op, x = _solved(problem)
    Is = float(np.sum(x @ lay.tab.I))
    h = 1e-5
    sgn = -1.0 if problem == INTERIOR else 1.0
    for p in _reflecting_points(lay, 4, 5 + problem):
        v = field.potential(lay, op, x, np.stack([p, (1 + sgn * h) * p, (1 + 2 * sgn * h) * p]))
        dvdn = sgn * (-3 * v[0] + 4 * v[1] - v[2]) / (2 * h)   # d/dr, the outward normal derivative
        want = -Is if problem == INTERIOR else 0.0
        assert abs(dvdn - want) < 1e-7 * abs(Is), (problem, dvdn, want)


def test_exterior_decay_at_infinity():
    # G_E(x, x') = 1/|x| + O(|x|^-2), so u(x) |x| -> I_sigma (flux 4 pi I_sigma at infinity)
    lay, op, x = _solved(EXTERIOR)
    Is = float(np.sum(x @ lay.tab.I))
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    gaps = []
    for R in (1e2, 1e3, 1e4):
        u = field.potential(lay, op, x, (R * d)[None, :])[0]
        gaps.append(abs(u * R - Is) / Is)
    assert gaps[1] < 0.2 * gaps[0] and gaps[2] < 0.2 * gaps[1] and gaps[2] < 1e-3, gaps


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_quadrature_converged_near_patches(problem):
    # targets eps/5 off the surface above patch points: 256 angles agree with 512
    lay, op, x = _solved(problem)
    g = np.random.default_rng(9)
    pts = []
    for i in range(lay.N):
        t, th = EPS * math.sqrt(g.random()), 2 * math.pi * g.random()
        p = system.patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], np.array([t]), np.array([th]))[0, 0]
        pts.append(p * (1 - EPS / 5 if problem == INTERIOR else 1 + EPS / 5))
    a = field.potential(lay, op, x, np.array(pts), ntheta=256)
    b = field.potential(lay, op, x, np.array(pts), ntheta=512)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_absorbing_condition_residual(problem):
    # the solved densities meet u = 1 (v = 1) on every patch: eq. l2res is at
    # the level of the discretisation; the physical field vanishes there; a
    # 1e-6 change of one coefficient shows in the residual
    lay, op, x = _solved(problem)
    for i in range(lay.N):
        res, r = field.l2_residual(lay, op, x, i, nt=8, ntheta=12)
        assert res < 1e-10, (i, res)
    t, th, _ = field.residual_grid(EPS, 4, 6)
    pts = system.patch_points(lay.c[:1], lay.e1[:1], lay.e2[:1], t, th)[0]
    phys = field.physical(lay, x, pts, field.potential(lay, op, x, pts))
    assert np.max(np.abs(phys)) < 1e-9
    xp = x.copy()
    xp[0, 0] *= 1 + 1e-6
    res_p, _ = field.l2_residual(lay, op, xp, 0, nt=8, ntheta=12)
    assert res_p > 100 * field.l2_residual(lay, op, x, 0, nt=8, ntheta=12)[0]
