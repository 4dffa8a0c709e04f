"""Compressed outgoing representation by interpolative decomposition (paper Section 7.1).

TEST INFRASTRUCTURE (oracle). FP64.

Steps as in the paper:
  1. Training grid x^t on the far-field region Theta = {arclength from the
     patch centre > 2 eps} (definition at the start of Section 7). Reading
     R13: rings at arclength r in [2 eps, pi), Chebyshev-distributed inside
     dyadic shells [2^j 2 eps, 2^(j+1) 2 eps], each ring with 2 n_theta
     equispaced azimuths (offset by half a step).
  2. A_jl = G(x_j^t, x_l^f) (n_t x n_f).
  3. ID of A, A ~ A[:, pi] Pi (eq. idapprox), computed the randomized way
     of Liberty et al. (cited for the ID): a Gaussian sketch Y = Omega A,
     column-pivoted QR of Y, rank p = #{|R_kk| > tol |R_11|}, and
     Pi = [I | R_11^-1 R_12] in pivot order.
  4. T = Pi W B (eq. Tmap); the skeleton is the fine-grid subset pi.

The Gaussian sketch is drawn from a fixed seed; it is part of this
precompute, not an input of the solver.
Pin (tests/test_oracle_id.py): at held-out points of Theta, the skeleton
field sum_m G(x, s_m) (T e_k)_m agrees with the full fine-grid quadrature
sum_l G(x, x_l^f) w_l B[l, k] for every basis function k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .greens import g_surface


def polar_to_xyz(t, theta):
    """Point at arclength t and angle theta about the north pole."""
    t = np.asarray(t, dtype=np.float64)
    theta = np.asarray(theta, dtype=np.float64)
    s = np.sin(t)
    return np.stack([s * np.cos(theta), s * np.sin(theta), np.cos(t)], axis=-1)


def training_grid(eps: float, ntheta_f: int, per_shell: int = 8):
    """Points of Theta (about the north pole) used to train the ID."""
    radii = [2.0 * eps]
    lo = 2.0 * eps
    rmax = math.pi * (1.0 - 1e-6)
    xc = np.cos((2 * np.arange(per_shell) + 1) * math.pi / (2 * per_shell))[::-1]
    while lo < rmax:
        hi = min(2.0 * lo, rmax)
        radii.extend(lo + 0.5 * (xc + 1.0) * (hi - lo))
        radii.append(hi)
        lo = hi
    radii = np.unique(np.array(radii))
    nth = 2 * ntheta_f
    th = 2.0 * math.pi * (np.arange(nth) + 0.5) / nth
    T = np.repeat(radii, nth)
    TH = np.tile(th, len(radii))
    return polar_to_xyz(T, TH)


@dataclass
class Compressed:
    T: np.ndarray          # (p, K)
    skel: np.ndarray       # (p,) indices into the fine grid
    skel_t: np.ndarray     # (p,) arclength of skeleton points
    skel_theta: np.ndarray # (p,) angle of skeleton points
    p: int
    tol: float
    n_train: int


def interpolative_decomposition(op, tol: float, seed: int = 12345, chunk: int = 2048
                                ) -> Compressed:
    """ID of A = G(x^t, x^f) for the one-patch result `op` (onepatch.OnePatch)."""
    xf = polar_to_xyz(op.fine_t, op.fine_theta)
    xt = training_grid(op.eps, op.ntheta)
    nt, nf = len(xt), len(xf)
    g = np.random.Generator(np.random.PCG64(seed))
    ell = min(nt, 1280)
    while True:
        Om = g.standard_normal((ell, nt))
        Y = np.empty((ell, nf))
        for c0 in range(0, nf, chunk):
            c1 = min(nf, c0 + chunk)
            diff = xt[:, None, :] - xf[None, c0:c1, :]
            d = np.sqrt(np.sum(diff * diff, axis=-1))
            Y[:, c0:c1] = Om @ g_surface(d, op.problem)
        Q, R, piv = sla.qr(Y, mode="economic", pivoting=True)
        diag = np.abs(np.diag(R))
        p = int(np.sum(diag > tol * diag[0]))
        if p < ell - 64 or ell >= nt:
            break
        ell = min(nt, 2 * ell)
    R11 = R[:p, :p]
    R12 = R[:p, p:]
    Tid = sla.solve_triangular(R11, R12)          # p x (nf - p)
    WB = op.w[:, None] * op.B                     # n_f x K
    T = WB[piv[:p], :] + Tid @ WB[piv[p:], :]     # T = Pi W B
    skel = piv[:p].copy()
    return Compressed(T, skel, op.fine_t[skel].copy(), op.fine_theta[skel].copy(), p, tol, nt)
