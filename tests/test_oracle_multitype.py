"""Pins of the oracle's several-radii system (oracle/multitype.py): the
single-radius system as a special case, compressed = uncompressed operator,
the absorbing condition on every patch of both radii, single-patch scalars."""
import math

import numpy as np
import pytest

import layouts
from oracle import multitype, system, tables
from oracle.greens import EXTERIOR, INTERIOR

pytestmark = pytest.mark.slow
RADII = (0.1, 0.05)
_FULL = {}


def _full(problem, eps):
    if (problem, eps) not in _FULL:
        from conftest import oracle_onepatch
        _FULL[(problem, eps)] = oracle_onepatch(problem, eps)
    return _FULL[(problem, eps)]


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_equal_radii_reduce_to_single_radius(problem):
    # two types with the same radius and tables: the single-radius system
    tab = tables.get(problem, 0.1, 15, 1e-12)
    c = layouts.uniform_centers(8, 0.1, 5)
    types = np.array([0, 1, 1, 0, 1, 0, 0, 1])
    lay = multitype.Layout(c, types, [tab, tab])
    ref = system.Layout(c, tab)
    x = layouts.random_coeffs(8, tab.K, 3, decay=0.1)
    assert np.max(np.abs(multitype.matvec_dense(lay, x) - system.matvec_dense(ref, x))) < 1e-14
    a, b = multitype.solve_dense(lay), system.solve_dense(ref)
    assert abs(a["I_sigma"] - b["I_sigma"]) < 1e-15
    assert np.max(np.abs(a["flux"] - b["flux"])) < 1e-15


def test_compressed_equals_uncompressed_two_radii():
    # the ID of each radius changes the operator only at the level of tol_id
    (t0, o0), (t1, o1) = _full(EXTERIOR, RADII[0]), _full(EXTERIOR, RADII[1])
    c, types = layouts.multi_radius_centers(4, RADII, 31)
    assert len(set(types.tolist())) == 2
    lay = multitype.Layout(c, types, [t0, t1])
    x = layouts.random_coeffs(4, t0.K, 5, decay=0.2)
    yc = multitype.matvec_dense(lay, x)
    yu = multitype.matvec_uncompressed(lay, [o0, o1], x)
    assert np.max(np.abs(yc - yu)) < 1e-10 * np.max(np.abs(yu - x))


def test_absorbing_condition_both_radii():
    """u = 1 on every patch of both radii at random off-grid points for the
    dense solution, to the discretisation level (degree-15 incoming fields;
    4e-10 on the two large patches of this layout that sit 0.32 apart, near
    their minimum separation 0.3; the same with the uncompressed operator's
    solution); a 1e-6 change of one coefficient shows."""
    (t0, o0), (t1, o1) = _full(EXTERIOR, RADII[0]), _full(EXTERIOR, RADII[1])
    c, types = layouts.multi_radius_centers(6, RADII, 44)
    lay = multitype.Layout(c, types, [t0, t1])
    x = multitype.solve_dense(lay)["x"]
    g = np.random.default_rng(2)
    for i in range(lay.N):
        eps = RADII[types[i]]
        t = eps * np.sqrt(g.random(12))
        th = 2 * np.pi * g.random(12)
        assert np.max(np.abs(multitype.patch_residual(lay, [o0, o1], x, i, t, th))) < 1e-9, i
    xp = x.copy()
    xp[0, 0] *= 1 + 1e-6
    assert np.max(np.abs(multitype.patch_residual(lay, [o0, o1], xp, 0, t, th))) > 1e-7


def test_single_patch_of_each_radius():
    t0 = tables.get(EXTERIOR, RADII[0], 15, 1e-12)
    t1 = tables.get(EXTERIOR, RADII[1], 15, 1e-12)
    for typ, tab in ((0, t0), (1, t1)):
        lay = multitype.Layout(np.array([[0.0, 0.6, 0.8]]), np.array([typ]), [t0, t1])
        r = multitype.solve_dense(lay)
        assert abs(r["capture_rate"] - 4 * math.pi * tab.I[0]) < 1e-15
    # a larger patch captures more
    assert t0.I[0] > t1.I[0]


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_field_equal_radii_reduces_to_single_radius(problem):
    # two types of one radius: the field is the single-radius one, at points
    # off the surface, on a patch and on the reflecting surface
    from oracle import field
    tab, op = _full(problem, RADII[0])
    c = layouts.uniform_centers(5, RADII[0], 71)
    types = np.array([0, 1, 0, 1, 1])
    lay = multitype.Layout(c, types, [tab, tab])
    ref = system.Layout(c, tab)
    x = layouts.random_coeffs(5, tab.K, 8, decay=0.1)
    r = 0.9 if problem == INTERIOR else 1.1
    g = np.random.default_rng(4)
    d = g.standard_normal((3, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    on = system.patch_points(c[1:2], ref.e1[1:2], ref.e2[1:2], np.array([0.04]), np.array([1.0]))[0]
    pts = np.vstack([r * d, on, d[:1]])
    a = multitype.potential(lay, [op, op], x, pts, ntheta=64)
    b = field.potential(ref, op, x, pts, ntheta=64)
    assert np.max(np.abs(a - b)) < 1e-14 * np.max(np.abs(b)), (a, b)


def test_field_absorbing_condition_and_flux_two_radii():
    """For the solved densities of two radii (interior): the field-based
    residual (eq. l2res, each patch's own radius) is at the discretisation
    level on patches of both radii, and dv/dn = -I_sigma on the reflecting
    surface (Section 2.3), by one-sided second-order differences."""
    (t0, o0), (t1, o1) = _full(INTERIOR, RADII[0]), _full(INTERIOR, RADII[1])
    c, types = layouts.multi_radius_centers(5, RADII, 52)
    assert len(set(types.tolist())) == 2
    lay = multitype.Layout(c, types, [t0, t1])
    sol = multitype.solve_dense(lay)
    x, Is = sol["x"], sol["I_sigma"]
    for i in (int(np.flatnonzero(types == 0)[0]), int(np.flatnonzero(types == 1)[0])):
        res, _ = multitype.l2_residual(lay, [o0, o1], x, i, nt=6, ntheta=10)
        assert res < 1e-8, (i, res)
    xp = x.copy()
    xp[0, 0] *= 1 + 1e-6
    assert multitype.l2_residual(lay, [o0, o1], xp, 0, nt=6, ntheta=10)[0] > 1e-6
    g = np.random.default_rng(6)
    h = 1e-5
    n_ok = 0
    while n_ok < 3:
        p = g.standard_normal(3)
        p /= np.linalg.norm(p)
        if np.min(np.arccos(np.clip(c @ p, -1, 1))) < 0.4:
            continue
        v = multitype.potential(lay, [o0, o1], x, np.stack([p, (1 - h) * p, (1 - 2 * h) * p]))
        dvdn = -(-3 * v[0] + 4 * v[1] - v[2]) / (2 * h)
        assert abs(dvdn + Is) < 1e-7 * abs(Is), (dvdn, -Is)
        n_ok += 1
