"""Scaled Zernike basis on a patch and the discrete Zernike transform (paper Section 4).

TEST INFRASTRUCTURE (oracle).

Readings (where the paper leaves the choice open):
  * basis order: n ascending; for each n, m = -n, -n+2, ..., n; negative m
    is the sin(|m| theta) function. K = (M+1)(M+2)/2.
  * q_k(t, theta) = Z_k(t/eps, theta) unnormalised (R_n^m(1) = 1); radial
    coordinate t = arclength from the patch centre.
  * sampling nodes: rho_a = the M+1 Gauss-Legendre nodes on [0,1] times the
    2M+2 equispaced angles theta_b = 2 pi b/(2M+2); K* = (M+1)(2M+2).
    Node index = a*(2M+2) + b.
  * P[k, (a,b)] = q_k(rho_a, theta_b) rho_a w_a (2 pi/(2M+2)) / ||Z_k||^2 with
    ||Z_n^m||^2 = (1 + delta_{m0}) pi / (2n + 2) (orthogonality relation
    eq. zorthog). The tensor rule integrates every product of two basis
    functions exactly, so P is the exact left inverse of synthesis on the span.

R_n^m follows the paper's Jacobi form R_n^m(r) = (-1)^((n-m)/2) r^m
P^{(m,0)}_{(n-m)/2}(1 - 2 r^2), using scipy's Jacobi polynomial.
Pins: tests/test_oracle_zernike.py (orthogonality, R(1)=1, P Q = I, P 1 = e_0,
explicit low-order polynomials).
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np
from scipy.special import eval_jacobi, roots_legendre


@lru_cache(maxsize=None)
def modes(M: int):
    """List of (n, m) in basis order (m < 0 is the sine function)."""
    out = []
    for n in range(M + 1):
        for m in range(-n, n + 1, 2):
            out.append((n, m))
    return tuple(out)


def nbasis(M: int) -> int:
    return (M + 1) * (M + 2) // 2


def radial(n: int, m: int, r):
    """Zernike radial polynomial R_n^|m|(r) in the paper's Jacobi form."""
    m = abs(m)
    if (n - m) % 2:
        raise ValueError("n - m must be even")
    s = (n - m) // 2
    r = np.asarray(r, dtype=np.float64)
    return (-1.0) ** s * r ** m * eval_jacobi(s, m, 0, 1.0 - 2.0 * r * r)


def basis(n: int, m: int, r, theta):
    """Z_n^m(r, theta): cos(m theta) for m >= 0, sin(|m| theta) for m < 0."""
    ang = np.cos(m * np.asarray(theta)) if m >= 0 else np.sin(-m * np.asarray(theta))
    return radial(n, m, r) * ang


def norm2(n: int, m: int) -> float:
    """Squared L2 norm on the unit disk with weight r (eq. zorthog)."""
    return (1.0 + (1.0 if m == 0 else 0.0)) * math.pi / (2 * n + 2)


@lru_cache(maxsize=None)
def nodes(M: int):
    """(rho (M+1,), w (M+1,), theta (2M+2,)): radial Gauss-Legendre on [0,1]
    and equispaced angles."""
    x, w = roots_legendre(M + 1)
    rho = 0.5 * (x + 1.0)
    wr = 0.5 * w
    nth = 2 * M + 2
    theta = 2.0 * math.pi * np.arange(nth) / nth
    return rho, wr, theta


def node_polar(M: int):
    """Flattened (rho, theta) of the K* sampling nodes, index a*(2M+2)+b."""
    rho, _, theta = nodes(M)
    R = np.repeat(rho, len(theta))
    T = np.tile(theta, len(rho))
    return R, T


def synthesis(M: int) -> np.ndarray:
    """Q_z (K* x K): basis functions sampled at the sampling nodes."""
    R, T = node_polar(M)
    return np.stack([basis(n, m, R, T) for (n, m) in modes(M)], axis=1)


def transform(M: int) -> np.ndarray:
    """Discrete Zernike transform P (K x K*)."""
    rho, wr, theta = nodes(M)
    nth = len(theta)
    R, T = node_polar(M)
    wq = np.repeat(rho * wr, nth) * (2.0 * math.pi / nth)
    rows = [basis(n, m, R, T) * wq / norm2(n, m) for (n, m) in modes(M)]
    return np.stack(rows, axis=0)
