"""Field of the patch densities at points of the domain, and the L2 residual
of the absorbing condition on a patch (paper Sections 2.2, 2.3 and 10).

TEST INFRASTRUCTURE (oracle). FP64, plain quadrature, small N only.

  potential      u(x) (exterior, eq. urep) or v(x) (interior, eq.
                 intBVPansatz): sum over every patch j of the integral of
                 G(x, x') sigma_j(x') over the patch, with sigma_j = B x_j
                 (Section 6), G the off-surface Neumann Green's function
                 (eqs. Gextoffsurface, Gintoffsurface). Every patch is
                 integrated by the one-patch solve's own radial rule (13
                 panels x 20 nodes, the Jacobi factor on the last) times
                 `ntheta` equispaced angles; sigma_j's angular dependence is
                 a trigonometric polynomial of degree M, so any ntheta > 2M
                 integrates it exactly against smooth data, and a larger one
                 resolves targets close to a patch. A target on the sphere
                 inside patch i takes patch i's term from the patch data
                 sum_k x_ik Z_k (what the one-patch solution reproduces on its
                 own patch, Section 9), the others by quadrature.
  physical       ubar = 1 - u (exterior, Section 2.2); vbar = (v - 1)/(3D) +
                 (1 - |x|^2)/6 with D = -I_sigma (eq. vtilde and the lemma
                 that follows it).
  l2_residual    (1/|Gamma_i|) ||v - 1||_{L2(Gamma_i)} on patch i (eq. l2res;
                 the normalisation as printed): Gauss-Legendre nodes in t on
                 [0, eps] times equispaced angles offset by half a step (a
                 grid that shares no point with the solve's), dS = sin t dt
                 dtheta, |Gamma_i| = 2 pi (1 - cos eps).

Pins (tests/test_oracle_field.py): v(0) = 2 I_sigma (G_I(0, x') = 2); the
normal derivative of v is -I_sigma and that of u is 0 on the reflecting
surface (the Neumann properties of Section 2.1, by finite differences);
u(x) |x| -> I_sigma as |x| -> infinity (G_E ~ 1/|x|, so the flux at
infinity is 4 pi I_sigma); convergence in ntheta at targets eps/5 off a
patch.
"""
from __future__ import annotations

import math

import numpy as np

from . import zernike
from .greens import EXTERIOR, INTERIOR, g_offsurface
from .system import patch_points


def _patch_quadrature(lay, op, x, j, ntheta):
    """Points (n_r * ntheta, 3) of patch j and sigma_j dS at them."""
    g = op.grid
    theta = 2.0 * math.pi * np.arange(ntheta) / ntheta
    pts = patch_points(lay.c[j:j + 1], lay.e1[j:j + 1], lay.e2[j:j + 1],
                       np.repeat(g.t, ntheta), np.tile(theta, len(g.t)))[0]
    sig = np.zeros((len(g.t), ntheta))
    for k, (n, m) in enumerate(zernike.modes(op.M)):
        ang = np.cos(m * theta) if m >= 0 else np.sin(-m * theta)
        sig += x[j, k] * np.outer(op.sigma[k], ang)
    w = (g.wsig * np.sin(g.t))[:, None] * (2.0 * math.pi / ntheta)
    return pts, (sig * w).ravel()


def on_patch(lay, point, tol: float = 1e-12):
    """Index of the patch containing `point` (on the sphere), or -1."""
    p = np.asarray(point, dtype=np.float64)
    if abs(np.linalg.norm(p) - 1.0) > tol:
        return -1
    ang = np.arctan2(np.linalg.norm(np.cross(lay.c, p), axis=1), lay.c @ p)
    i = int(np.argmin(ang))
    return i if ang[i] <= lay.tab.eps * (1 + tol) else -1


def self_term(lay, x, i, point):
    """sum_k x_ik Z_k(t/eps, theta) at a point of patch i."""
    p = np.asarray(point, dtype=np.float64)
    t = math.atan2(np.linalg.norm(np.cross(lay.c[i], p)), float(lay.c[i] @ p))
    th = math.atan2(float(lay.e2[i] @ p), float(lay.e1[i] @ p))
    r = min(t / lay.tab.eps, 1.0)
    return sum(x[i, k] * float(zernike.basis(n, m, r, th)) for k, (n, m) in enumerate(zernike.modes(lay.tab.M)))


def potential(lay, op, x, points, ntheta: int = 256):
    """u (exterior) or v (interior) at each of `points` (n, 3)."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    prob = lay.tab.problem
    quad = [_patch_quadrature(lay, op, x, j, ntheta) for j in range(lay.N)]
    out = np.zeros(len(points))
    for a, p in enumerate(points):
        i = on_patch(lay, p)
        for j in range(lay.N):
            if j == i:
                out[a] += self_term(lay, x, i, p)
            else:
                pts, sw = quad[j]
                out[a] += float(np.sum(g_offsurface(p[None, :], pts, prob) * sw))
    return out


def physical(lay, x, points, pot):
    """ubar = 1 - u (exterior); vbar = (v - 1)/(3 D) + (1 - |x|^2)/6, D = -I_sigma (interior)."""
    if lay.tab.problem == EXTERIOR:
        return 1.0 - pot
    Is = float(np.sum(x @ lay.tab.I))
    r2 = np.sum(np.atleast_2d(points) ** 2, axis=1)
    return (pot - 1.0) / (3.0 * -Is) + (1.0 - r2) / 6.0


def residual_grid(eps: float, nt: int, ntheta: int):
    """(t, theta, weight) of the residual rule on a patch: Gauss-Legendre in t on
    [0, eps] times ntheta angles offset by half a step; weight = dt dtheta sin t."""
    xg, wg = np.polynomial.legendre.leggauss(nt)
    t = 0.5 * eps * (xg + 1.0)
    wt = 0.5 * eps * wg * np.sin(t)
    th = 2.0 * math.pi * (np.arange(ntheta) + 0.5) / ntheta
    return np.repeat(t, ntheta), np.tile(th, nt), np.repeat(wt, ntheta) * (2.0 * math.pi / ntheta)


def l2_residual(lay, op, x, i: int, nt: int = 20, ntheta: int = 40, ntheta_quad: int = 256):
    """(1/|Gamma_i|) ||v - 1||_{L2(Gamma_i)} on patch i (eq. l2res)."""
    t, th, w = residual_grid(lay.tab.eps, nt, ntheta)
    pts = patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], t, th)[0]
    r = potential(lay, op, x, pts, ntheta_quad) - 1.0
    area = 2.0 * math.pi * (1.0 - math.cos(lay.tab.eps))
    return math.sqrt(float(np.sum(w * r * r))) / area, r
