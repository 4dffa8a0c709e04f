"""Pins of the oracle's sphere Neumann Green's functions (paper Section 2.1)."""
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle.greens import EXTERIOR, INTERIOR, g_offsurface, g_points, g_surface


def _unit(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


@pytest.fixture(scope="module")
def pts():
    g = np.random.Generator(np.random.PCG64(11))
    x = _unit(g.standard_normal((200, 3)))
    xp = _unit(g.standard_normal((200, 3)))
    return x, xp


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_surface_form_equals_general_form(pts, problem):
    # eqs. Gextonsurface / Gintonsurface are the restrictions of
    # eqs. Gextoffsurface / Gintoffsurface to |x| = 1.
    x, xp = pts
    d = np.linalg.norm(x - xp, axis=1)
    a = g_surface(d, problem)
    b = g_offsurface(x, xp, problem)
    assert np.max(np.abs(a - b) / np.abs(a)) < 1e-13


@pytest.mark.parametrize("problem,expected", [(EXTERIOR, 0.0), (INTERIOR, -1.0)])
def test_normal_derivative_on_sphere(pts, problem, expected):
    # dG/dn = 0 (exterior) and -1 (interior) on the sphere away from the
    # source (eqs. Gextproperties, Gintproperties; by symmetry of G the
    # derivative may be taken in either argument).
    x, xp = pts
    h = 1e-5
    if problem == EXTERIOR:
        fp = g_offsurface(x * (1 + 2 * h), xp, problem)
        f0 = g_offsurface(x * (1 + h), xp, problem)
        f1 = g_offsurface(x, xp, problem)
        deriv = (-3 * f1 + 4 * f0 - fp) / (2 * h)      # one-sided, radius >= 1
    else:
        fm = g_offsurface(x * (1 - 2 * h), xp, problem)
        f0 = g_offsurface(x * (1 - h), xp, problem)
        f1 = g_offsurface(x, xp, problem)
        deriv = (3 * f1 - 4 * f0 + fm) / (2 * h)       # one-sided, radius <= 1
    assert np.max(np.abs(deriv - expected)) < 2e-6


@pytest.mark.parametrize("problem,sign", [(INTERIOR, -1.0), (EXTERIOR, 1.0)])
def test_harmonic_off_the_sphere(problem, sign):
    # -Laplace G = 4 pi delta: away from the source the general form is harmonic.
    g = np.random.Generator(np.random.PCG64(5))
    xp = _unit(g.standard_normal((50, 3)))
    x = _unit(g.standard_normal((50, 3))) * (1.0 + sign * 0.3)
    def lap(h):
        out = -6.0 * g_offsurface(x, xp, problem)
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            out += g_offsurface(x + e, xp, problem) + g_offsurface(x - e, xp, problem)
        return out / (h * h)
    coarse, fine = np.abs(lap(1e-2)), np.abs(lap(1e-3))
    # second-order stencil: the residual must vanish like h^2
    assert np.max(fine) < 1e-3
    assert np.max(fine) < 0.02 * np.max(coarse)


def test_interior_value_at_centre():
    # G_I(0, x') = 2 for |x'| = 1 (used in the proof that I_sigma != 0).
    g = np.random.Generator(np.random.PCG64(3))
    xp = _unit(g.standard_normal((20, 3)))
    assert np.allclose(g_offsurface(np.zeros((20, 3)), xp, INTERIOR), 2.0, atol=1e-14)


@pytest.mark.parametrize("problem,mean", [(INTERIOR, 2.0), (EXTERIOR, 1.0)])
def test_sphere_mean(problem, mean):
    # (1/4 pi) int G(x, x') dS(x) = 2 for G_I (Section 2.3) and 1 for G_E:
    # on the sphere dS = 2 pi d dd in the chord d, so the mean is (1/2) int_0^2 G d dd.
    val, err = quad(lambda d: 0.5 * g_surface(d, problem) * d, 0.0, 2.0,
                    epsabs=1e-15, epsrel=1e-15, limit=200)
    assert abs(val - mean) < 1e-13


def test_symmetry_bitwise(pts):
    x, xp = pts
    for problem in (INTERIOR, EXTERIOR):
        a = g_points(x, xp, problem)
        b = g_points(xp, x, problem)
        assert np.array_equal(a, b)
