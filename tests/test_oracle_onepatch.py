"""Pins of the oracle's one-patch solver (paper Sections 5 and 9)."""
import math

import numpy as np
import pytest
from scipy.special import ellipe, ellipkm1, roots_legendre, gamma

from oracle import onepatch as op
from oracle import zernike
from oracle.greens import EXTERIOR, INTERIOR, g_surface


# ------------------------------------------------------------ modal kernels
def _legendre_q_form(t, tp, M):
    """G^(1)_m = 2 Q_{m-1/2}(chi) / (pi sqrt(sin t sin t')) with the toroidal
    Legendre functions from complete elliptic integrals and the upward
    three-term recurrence (stable for chi close to 1)."""
    cm1 = 2 * np.sin((t - tp) / 2) ** 2 / (np.sin(t) * np.sin(tp))   # chi - 1, no cancellation
    chi = 1 + cm1
    k2 = 2 / (chi + 1)
    k = np.sqrt(k2)
    K = ellipkm1(cm1 / (chi + 1))
    E = ellipe(k2)
    Q = np.empty((len(tp), M + 1))
    Q[:, 0] = k * K
    Q[:, 1] = chi * k * K - (2 / k) * E
    for m in range(1, M):
        Q[:, m + 1] = (2 * m * chi * Q[:, m] - (m - 0.5) * Q[:, m - 1]) / (m + 0.5)
    return 2 / math.pi * Q / np.sqrt(np.sin(t) * np.sin(tp))[:, None]


def test_modal_g2_closed_form():
    # Section 9.1: (1/pi) int log(2/d) cos(n phi) = -log(cos(t1/2) sin(t2/2)) (n = 0),
    # (tan(t1/2) cot(t2/2))^n / (2n) (n > 0)
    eps = 0.1
    t = 0.37 * eps
    tp = np.array([0.36, 0.30, 0.5, 0.9, 0.05, 0.3701, 0.99]) * eps
    _, G2, _ = op.modal_pieces(t, tp, 15)
    t1, t2 = np.minimum(t, tp), np.maximum(t, tp)
    ref = np.empty_like(G2)
    ref[:, 0] = -np.log(np.cos(t1 / 2) * np.sin(t2 / 2))
    for n in range(1, 16):
        ref[:, n] = (np.tan(t1 / 2) / np.tan(t2 / 2)) ** n / (2 * n)
    assert np.max(np.abs(G2 - ref)) < 1e-13


def test_modal_g1_legendre_functions():
    # Heine's toroidal identity: (1/pi) int_0^pi cos(m phi)/|x-x'| dphi = Q_{m-1/2}(chi)/(pi sqrt(r r'))
    eps = 0.05
    t = 0.61 * eps
    tp = np.array([0.6, 0.62, 0.55, 0.6100001, 0.6099, 0.7]) * eps
    G1, _, _ = op.modal_pieces(t, tp, 15)
    ref = _legendre_q_form(t, tp, 15)
    assert np.max(np.abs(G1 - ref) / np.abs(ref).max(axis=1, keepdims=True)) < 1e-13


@pytest.mark.parametrize("problem", [INTERIOR, EXTERIOR])
def test_modal_fourier_series_reproduces_kernel(problem):
    # G(d(t,t',phi)) = G_0 + 2 sum_m G_m cos(m phi) at well-separated t, t'
    # (the modes decay like (t/t')^m, so m <= 15 suffices at t/t' < 0.09)
    eps = 0.1
    t, tp = 0.08 * eps, np.array([0.95 * eps])
    M = 15
    Gm = op.modal_kernel(t, tp, M, problem)[0]
    for phi in (0.0, 0.7, 2.0, math.pi):
        d = math.sqrt(2 * (1 - math.cos(t) * math.cos(tp[0])
                           - math.sin(t) * math.sin(tp[0]) * math.cos(phi)))
        series = Gm[0] + 2 * np.sum(Gm[1:] * np.cos(np.arange(1, M + 1) * phi))
        assert abs(series - g_surface(d, problem)) < 1e-12 * abs(g_surface(d, problem))


def test_quadrature_rules_exact_moments():
    x, w = op._gl(20)
    for k in range(0, 40):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x**k) - exact) < 1e-14
    # Gauss-Jacobi for (1-x)^(-1/2): int_{-1}^1 (1-x)^(-1/2) (1+x)^k dx = 2^(k+1/2) B(1/2, k+1)
    xj, wj = op._gj(20)
    for k in range(0, 40):
        exact = 2 ** (k + 0.5) * gamma(0.5) * gamma(k + 1) / gamma(k + 1.5)
        assert abs(np.sum(wj * (1 + xj) ** k) - exact) < 1e-13 * exact


def test_panel_breaks():
    a = op.panel_breaks(1.0)
    assert a[0] == 0 and a[1] == 0.5 and a[2] == 0.75 and a[-1] == 1.0 and len(a) == 14
    assert abs(a[12] - (1 - 2**-12)) < 1e-16


# ------------------------------------------------------------ one-patch solution
@pytest.fixture(scope="module")
def patch_e():
    return op.solve_one_patch(0.1, EXTERIOR, M=15)


def _polar_potential(res, k, tstar, thstar, npsi=160, nq=30):
    """int_Gamma G(x*, x') b_k(x') dS(x') by a 2-D quadrature in geodesic
    polar coordinates (rho, psi) about x*: dS = sin rho drho dpsi, which
    cancels the 2/d singularity. The rho integral is split where the ray
    crosses the panel circles and ends at the patch edge with rho = rho_max - s^2
    (square-root edge behaviour); psi uses the trapezoidal rule."""
    eps, problem = res.eps, res.problem
    n, m = zernike.modes(res.M)[k]
    xs = np.array([math.sin(tstar) * math.cos(thstar), math.sin(tstar) * math.sin(thstar),
                   math.cos(tstar)])
    u1 = np.array([math.cos(tstar) * math.cos(thstar), math.cos(tstar) * math.sin(thstar),
                   -math.sin(tstar)])
    u2 = np.array([-math.sin(thstar), math.cos(thstar), 0.0])
    xg, wg = roots_legendre(nq)
    total = 0.0
    breaks = op.panel_breaks(eps)
    for ip in range(npsi):
        psi = 2 * math.pi * ip / npsi
        A, B = math.cos(tstar), -math.sin(tstar) * math.cos(psi)
        R, dl = math.hypot(A, B), math.atan2(B, A)
        rmax = dl + math.acos(math.cos(eps) / R)
        cuts = [0.0, rmax]
        for a in breaks[1:-1]:
            c = math.cos(a) / R
            if c <= 1.0:
                for r in (dl + math.acos(c), dl - math.acos(c)):
                    if 1e-14 < r < rmax - 1e-14:
                        cuts.append(r)
        cuts = sorted(cuts)
        if len(cuts) == 2:
            cuts = [0.0, 0.5 * rmax, rmax]
        nodes, wts = [], []
        # first piece: graded toward rho = 0 (rho log rho behaviour)
        lo, hi = cuts[0], cuts[1]
        edges = [hi * 2.0 ** (-j) for j in range(45, -1, -1)]
        edges = [0.0] + edges
        for a, b in zip(edges[:-1], edges[1:]):
            nodes.append(a + 0.5 * (b - a) * (xg + 1))
            wts.append(0.5 * (b - a) * wg)
        for a, b in zip(cuts[1:-2], cuts[2:-1]):
            nodes.append(a + 0.5 * (b - a) * (xg + 1))
            wts.append(0.5 * (b - a) * wg)
        # last piece: rho = rmax - s^2
        a = cuts[-2]
        smax = math.sqrt(rmax - a)
        s = 0.5 * smax * (xg + 1)
        nodes.append(rmax - s * s)
        wts.append(0.5 * smax * wg * 2 * s)
        rho = np.concatenate(nodes)
        w = np.concatenate(wts)
        dirv = math.cos(psi) * u1 + math.sin(psi) * u2
        xp = np.cos(rho)[:, None] * xs[None, :] + np.sin(rho)[:, None] * dirv[None, :]
        tp = np.arctan2(np.hypot(xp[:, 0], xp[:, 1]), xp[:, 2])
        tp = np.minimum(tp, eps * (1 - 1e-15))
        thp = np.arctan2(xp[:, 1], xp[:, 0])
        sig = op.sigma_at(res, k, tp)
        ang = np.cos(m * thp) if m >= 0 else np.sin(-m * thp)
        d = 2 * np.sin(rho / 2)
        f = g_surface(d, problem) * sig * ang * np.sin(rho)
        total += np.sum(w * f)
    return total * 2 * math.pi / npsi


@pytest.mark.slow
def test_one_patch_residual_off_grid(patch_e):
    # Section 9.3: the computed b_k solves S b_k = q_k at points that are not
    # collocation nodes (residual measured by an independent quadrature).
    res = patch_e
    modes = zernike.modes(15)
    for k in (0, modes.index((3, 1)), modes.index((8, -4)), modes.index((15, 15))):
        n, m = modes[k]
        for ts, th in ((0.137, 0.3), (0.55, 2.1), (0.93, 4.0)):
            tstar = ts * res.eps
            val = _polar_potential(res, k, tstar, th)
            ref = zernike.basis(n, m, ts, th)
            # the polar rule itself stalls near 1e-9 for targets near the
            # edge (rays nearly tangent to the rim); it converges further inside
            tol = 1e-9 if ts < 0.6 else 3e-9
            assert abs(val - ref) < tol, (k, ts, val, ref)


def test_flat_disk_limit_and_sign():
    # As eps -> 0 the patch becomes a flat disk; for the kernel 2/|x - x'| the
    # total charge at unit potential is eps/pi (Weber disk), so I_0 pi / eps -> 1.
    # The log(2/d) term enters G_I with + and G_E with -, so the interior
    # charge is below and the exterior charge above the flat value, with a gap
    # of order eps log(1/eps).
    gaps = {}
    for eps in (0.03, 0.003):
        for problem in (INTERIOR, EXTERIOR):
            grid = op.radial_grid(eps)
            A0 = op.modal_matrices(grid, 0, problem)[0]
            sig = np.linalg.solve(A0, np.ones(len(grid.t)))
            I0 = 2 * math.pi * np.sum(grid.wsig * np.sin(grid.t) * sig)
            gaps[(eps, problem)] = I0 * math.pi / eps - 1
    for eps in (0.03, 0.003):
        assert gaps[(eps, INTERIOR)] < 0 < gaps[(eps, EXTERIOR)]
        lead = eps / math.pi * math.log(2 / eps)
        assert 0.5 * lead < abs(gaps[(eps, INTERIOR)]) < 2 * lead
        assert 0.5 * lead < abs(gaps[(eps, EXTERIOR)]) < 2 * lead
    assert abs(gaps[(0.003, INTERIOR)]) < 0.25 * abs(gaps[(0.03, INTERIOR)])


def test_I_vector_structure(patch_e):
    # I = w^T B: only the m = 0 basis functions have non-zero integrals.
    modes = zernike.modes(15)
    for k, (n, m) in enumerate(modes):
        if m != 0:
            assert abs(patch_e.I[k]) < 1e-15
    assert patch_e.I[0] > 0
