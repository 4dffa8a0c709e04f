"""Pins of the oracle's Zernike basis and discrete transform (paper Section 4)."""
import math

import numpy as np
import pytest
from scipy.special import roots_legendre

from oracle import zernike as z


def test_count():
    assert z.nbasis(15) == 136 == len(z.modes(15))


def test_radial_is_one_at_edge():
    assert max(abs(z.radial(n, m, 1.0) - 1.0) for n, m in z.modes(15)) < 1e-13


def test_textbook_radial_polynomials():
    r = np.linspace(0, 1, 17)
    assert np.allclose(z.radial(2, 0, r), 2 * r**2 - 1, atol=1e-14)
    assert np.allclose(z.radial(4, 0, r), 6 * r**4 - 6 * r**2 + 1, atol=1e-14)
    assert np.allclose(z.radial(3, 1, r), 3 * r**3 - 2 * r, atol=1e-14)
    assert np.allclose(z.radial(4, 2, r), 4 * r**4 - 3 * r**2, atol=1e-14)
    assert np.allclose(z.radial(5, 1, r), 10 * r**5 - 12 * r**3 + 3 * r, atol=1e-14)


def test_orthogonality_constants():
    # eq. zorthog with an independent, larger tensor rule
    M = 15
    x, w = roots_legendre(40)
    r = 0.5 * (x + 1)
    wr = 0.5 * w
    nth = 97
    th = 2 * math.pi * np.arange(nth) / nth
    R = np.repeat(r, nth)
    T = np.tile(th, len(r))
    W = np.repeat(r * wr, nth) * 2 * math.pi / nth
    F = np.stack([z.basis(n, m, R, T) for n, m in z.modes(M)], axis=1)
    G = F.T @ (W[:, None] * F)
    D = np.diag([z.norm2(n, m) for n, m in z.modes(M)])
    assert np.max(np.abs(G - D)) < 1e-13


def test_transform_left_inverse_and_constant():
    M = 15
    P = z.transform(M)
    Q = z.synthesis(M)
    assert P.shape == (136, 512)
    assert np.max(np.abs(P @ Q - np.eye(136))) < 1e-12
    e0 = P @ np.ones(512)
    assert abs(e0[0] - 1) < 1e-14 and np.max(np.abs(e0[1:])) < 1e-13
