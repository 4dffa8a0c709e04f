"""Many-patch multiple scattering system, its solution, and the scalars (paper Sections 3, 6, 8, 2).

TEST INFRASTRUCTURE (oracle). FP64.

  frames           per-patch polar frame (reading R5: theta = 0 along the
                   projection of z-hat, or of x-hat when |c.z| > 1/sqrt 2)
  patch_points     x = cos t c + sin t (cos theta e1 + sin theta e2): the
                   one-patch parametrisation of Section 9 rotated to c
  matvec_dense     y_i = x_i + P sum_{j != i} G(Z_i, S_j) (T x_j)
                   (eq. opinteqnsdisc with S_ij B replaced by its compressed
                   form G(., S_j) T, eqs. outgoingcompressed and Tmap)
  matvec_uncompressed
                   y_i = x_i + P sum_{j != i} S_ij B x_j, S_ij(k, l) =
                   G(z_ik, x^f_jl) w_l (eq. Sijquad; small N only)
  dense_matrix     the KN x KN matrix of the compressed system (small N)
  gmres            unrestarted GMRES, modified Gram-Schmidt, x0 = 0
  scalars          I_sigma = I . sum_i x_i (eq. getI); mu = 1/(3 I_sigma) - 3/5
                   (eq. mufromsigma2); exterior: I_sigma, the paper's
                   J = -I_sigma, and the capture rate 4 pi I_sigma (reading R1);
                   per-patch flux I . x_i
The right-hand side is P 1 = e_0 on every patch (1 = Z_0^0).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np

from . import zernike
from .greens import EXTERIOR, INTERIOR, g_surface


def frames(c: np.ndarray):
    """(e1, e2) for unit centres c (N x 3), reading R5."""
    c = np.asarray(c, dtype=np.float64)
    a = np.zeros_like(c)
    use_x = np.abs(c[:, 2]) > 1.0 / math.sqrt(2.0)
    a[~use_x, 2] = 1.0
    a[use_x, 0] = 1.0
    e1 = a - np.sum(a * c, axis=1, keepdims=True) * c
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(c, e1)
    return e1, e2


def patch_points(c, e1, e2, t, theta):
    """Points (N, n, 3) at polar coordinates (t, theta) (length n) on each patch."""
    ct = np.cos(t)[None, :, None]
    st = np.sin(t)[None, :, None]
    cth = np.cos(theta)[None, :, None]
    sth = np.sin(theta)[None, :, None]
    return (ct * c[:, None, :] + st * (cth * e1[:, None, :] + sth * e2[:, None, :]))


@dataclass
class Tables:
    """Per-(problem, eps, M) precompute outputs used by the matvec."""
    problem: int
    eps: float
    M: int
    T: np.ndarray          # (p, K)
    skel_t: np.ndarray     # (p,)
    skel_theta: np.ndarray # (p,)
    I: np.ndarray          # (K,)
    P: np.ndarray          # (K, K*)
    node_t: np.ndarray     # (K*,) arclength of Zernike nodes = eps * rho
    node_theta: np.ndarray # (K*,)

    @property
    def K(self):
        return self.T.shape[1]

    @property
    def p(self):
        return self.T.shape[0]


class Layout:
    """Patch centres plus derived point sets."""

    def __init__(self, centers: np.ndarray, tab: Tables):
        self.c = np.asarray(centers, dtype=np.float64)
        self.N = len(self.c)
        self.e1, self.e2 = frames(self.c)
        self.tab = tab
        self.Z = patch_points(self.c, self.e1, self.e2, tab.node_t, tab.node_theta)
        self.S = patch_points(self.c, self.e1, self.e2, tab.skel_t, tab.skel_theta)


def green_block(X, Y, problem):
    diff = X[:, None, :] - Y[None, :, :]
    d = np.sqrt(np.sum(diff * diff, axis=-1))
    return g_surface(d, problem)


def incoming_dense(lay: Layout, x: np.ndarray, targets=None) -> np.ndarray:
    """U_i = sum_{j != i} G(Z_i, S_j) (T x_j) at the K* nodes of each target
    patch (the scattered field before projection)."""
    tab = lay.tab
    rho = x @ tab.T.T                                 # (N, p) outgoing strengths
    tl = range(lay.N) if targets is None else targets
    U = np.zeros((len(tl), lay.Z.shape[1]))
    for a, i in enumerate(tl):
        for j in range(lay.N):
            if j != i:
                U[a] += green_block(lay.Z[i], lay.S[j], tab.problem) @ rho[j]
    return U


def matvec_dense(lay: Layout, x: np.ndarray, incoming: Optional[Callable] = None
                 ) -> np.ndarray:
    """Compressed system matrix applied to x (N x K)."""
    U = incoming_dense(lay, x) if incoming is None else incoming(lay, x)
    return x + U @ lay.tab.P.T


def matvec_uncompressed(lay: Layout, op, x: np.ndarray) -> np.ndarray:
    """Uncompressed system (S_ij B with the full fine grid), for small N.
    `op` is the onepatch.OnePatch of the same (problem, eps, M)."""
    tab = lay.tab
    Xf = patch_points(lay.c, lay.e1, lay.e2, op.fine_t, op.fine_theta)
    sig_w = (x @ op.B.T) * op.w[None, :]               # (N, n_f): sigma_j w
    y = x.copy()
    for i in range(lay.N):
        u = np.zeros(lay.Z.shape[1])
        for j in range(lay.N):
            if j != i:
                u += green_block(lay.Z[i], Xf[j], tab.problem) @ sig_w[j]
        y[i] += tab.P @ u
    return y


def dense_matrix(lay: Layout) -> np.ndarray:
    """KN x KN compressed system matrix: identity blocks on the diagonal and
    P G(Z_i, S_j) T off it."""
    tab = lay.tab
    K, N = tab.K, lay.N
    A = np.eye(K * N)
    for i in range(N):
        for j in range(N):
            if j != i:
                A[i * K:(i + 1) * K, j * K:(j + 1) * K] = (
                    tab.P @ green_block(lay.Z[i], lay.S[j], tab.problem) @ tab.T)
    return A


def rhs(N: int, K: int) -> np.ndarray:
    b = np.zeros((N, K))
    b[:, 0] = 1.0
    return b


def gmres(apply: Callable[[np.ndarray], np.ndarray], b: np.ndarray, tol: float,
          maxiter: int = 500, x0: Optional[np.ndarray] = None):
    """Unrestarted GMRES (modified Gram-Schmidt, Givens rotations), stopping
    on ||b - A x||_2 / ||b||_2 <= tol. Returns (x, iterations, residual history)."""
    shape = b.shape
    bv = b.ravel()
    x = np.zeros_like(bv) if x0 is None else x0.ravel().copy()
    r = bv - apply(x.reshape(shape)).ravel() if x0 is not None else bv.copy()
    bnorm = np.linalg.norm(bv)
    beta = np.linalg.norm(r)
    hist = [beta / bnorm]
    if beta / bnorm <= tol:
        return x.reshape(shape), 0, hist
    V = [r / beta]
    H = np.zeros((maxiter + 1, maxiter))
    cs = np.zeros(maxiter)
    sn = np.zeros(maxiter)
    g = np.zeros(maxiter + 1)
    g[0] = beta
    k = 0
    for k in range(maxiter):
        w = apply(V[k].reshape(shape)).ravel()
        for j in range(k + 1):
            H[j, k] = w @ V[j]
            w = w - H[j, k] * V[j]
        hk1 = np.linalg.norm(w)
        H[k + 1, k] = hk1
        for j in range(k):
            a, bb = H[j, k], H[j + 1, k]
            H[j, k] = cs[j] * a + sn[j] * bb
            H[j + 1, k] = -sn[j] * a + cs[j] * bb
        den = math.hypot(H[k, k], H[k + 1, k])
        cs[k], sn[k] = H[k, k] / den, H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / bnorm)
        if hist[-1] <= tol or hk1 == 0.0:
            break
        V.append(w / hk1)
    n = k + 1
    y = np.linalg.solve(np.triu(H[:n, :n]), g[:n])
    for j in range(n):
        x = x + y[j] * V[j]
    return x.reshape(shape), n, hist


def scalars(tab: Tables, x: np.ndarray) -> dict:
    """I_sigma and the problem's scalar output."""
    flux = x @ tab.I
    Is = float(np.sum(flux))
    out = {"I_sigma": Is, "flux": flux}
    if tab.problem == INTERIOR:
        out["mu"] = 1.0 / (3.0 * Is) - 0.6
    else:
        out["J_paper"] = -Is
        out["capture_rate"] = 4.0 * math.pi * Is
    return out


def solve_dense(lay: Layout) -> dict:
    """Dense LU solve of the compressed system (small N)."""
    A = dense_matrix(lay)
    b = rhs(lay.N, lay.tab.K).ravel()
    x = np.linalg.solve(A, b).reshape(lay.N, lay.tab.K)
    out = scalars(lay.tab, x)
    out["x"] = x
    return out


def solve_gmres(lay: Layout, tol: float = 1e-12, maxiter: int = 300, incoming=None) -> dict:
    b = rhs(lay.N, lay.tab.K)
    x, it, hist = gmres(lambda v: matvec_dense(lay, v, incoming), b, tol, maxiter)
    out = scalars(lay.tab, x)
    out.update(x=x, iters=it, hist=hist)
    return out


def patch_residual(lay: Layout, op, x: np.ndarray, i: int, t: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """v - 1 at points (t, theta) of patch i, v = sum_j S_j[sigma_j] the
    single-layer potential of the densities sigma_j = B x_j (Sections 3 and 6):
    the self term is the patch's data sum_k x_ik Z_k (what the one-patch solve
    reproduces on its own patch), the other patches' terms come from the fine
    quadrature of their densities. Zero up to the truncation of the incoming
    fields to degree M when x solves the system; the paper's L2 residual error
    on a patch (eq. patcherrl2, Sections 9.3 and 10.2) is its root mean square."""
    tab = lay.tab
    self_part = np.zeros(len(t))
    for k, (n, m) in enumerate(zernike.modes(tab.M)):
        self_part += x[i, k] * zernike.basis(n, m, t / tab.eps, theta)
    X = patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], t, theta)[0]
    far = np.zeros(len(t))
    for j in range(lay.N):
        if j != i:
            Xf = patch_points(lay.c[j:j + 1], lay.e1[j:j + 1], lay.e2[j:j + 1], op.fine_t, op.fine_theta)[0]
            far += green_block(X, Xf, tab.problem) @ ((op.B @ x[j]) * op.w)
    return self_part + far - 1.0

