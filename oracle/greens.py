"""Neumann Green's functions of the unit sphere (paper Section 2.1).

TEST INFRASTRUCTURE (oracle). FP64, written out directly from the paper's
closed forms.

  exterior, source on the sphere   eq. (Gextoffsurface)
  exterior, both on the sphere     eq. (Gextonsurface)
  interior, source on the sphere   eq. (Gintoffsurface)
  interior, both on the sphere     eq. (Gintonsurface)

problem = 0 means interior (narrow escape), 1 exterior (narrow capture).
Pins: tests/test_oracle_greens.py (surface forms vs the general forms,
normal derivatives 0 and -1, G_I(0, x') = 2, sphere means, symmetry).
"""
from __future__ import annotations

import numpy as np

INTERIOR = 0
EXTERIOR = 1


def g_surface(d, problem: int):
    """G(x, x') for |x| = |x'| = 1 as a function of the chord d = |x - x'|.

    exterior: 2/d - log(2/d) - log(1 + d/2)      (Gextonsurface)
    interior: 2/d + log(2/d) - log(1 + d/2)      (Gintonsurface)
    """
    d = np.asarray(d, dtype=np.float64)
    if problem == EXTERIOR:
        return 2.0 / d - np.log(2.0 / d) - np.log1p(0.5 * d)
    if problem == INTERIOR:
        return 2.0 / d + np.log(2.0 / d) - np.log1p(0.5 * d)
    raise ValueError(problem)


def g_offsurface(x, xp, problem: int):
    """G(x, x') for x' on the sphere and x anywhere off it (|x|>=1 exterior,
    |x|<=1 interior), from the paper's general forms.

    exterior: 2/|x-x'| + log((|x| - x.x') / (1 - x.x' + |x-x'|))   (Gextoffsurface)
    interior: 2/|x-x'| + log(2 / (1 - x.x' + |x-x'|))              (Gintoffsurface)
    """
    x = np.asarray(x, dtype=np.float64)
    xp = np.asarray(xp, dtype=np.float64)
    diff = x - xp
    r = np.sqrt(np.sum(diff * diff, axis=-1))
    dot = np.sum(x * xp, axis=-1)
    if problem == EXTERIOR:
        nx = np.sqrt(np.sum(x * x, axis=-1))
        return 2.0 / r + np.log((nx - dot) / (1.0 - dot + r))
    if problem == INTERIOR:
        return 2.0 / r + np.log(2.0 / (1.0 - dot + r))
    raise ValueError(problem)


def g_points(x, xp, problem: int):
    """Surface Green's function between two point sets on the sphere.

    x: (..., 3), xp: (..., 3) broadcastable; the chord is formed from
    coordinate differences (never from sqrt(2 - 2 x.x'))."""
    diff = np.asarray(x) - np.asarray(xp)
    d = np.sqrt(np.sum(diff * diff, axis=-1))
    return g_surface(d, problem)
