"""Several patch radii in one configuration (the paper's Section 11 names
patches of different sizes as an extension; Sections 3, 6 and 8 carry over
with one precompute per patch radius).

TEST INFRASTRUCTURE (oracle). FP64, dense, small N.

Patch i has type tau_i with radius eps_tau and that radius's one-patch
tables (T_tau, skeleton, I_tau; P is the same for every radius, since it acts
on the scaled Zernike functions of t/eps). The system (eq. opinteqnsdisc with
per-patch operators) is

    f_i + P sum_{j != i} G(Z_i, S_j) T_{tau_j} f_j = e_0,

Z_i the sampling nodes of patch i (arclength eps_{tau_i} rho), S_j the skeleton
of patch j's type. Scalars: I_sigma = sum_i I_{tau_i} . f_i, then mu and the
capture rate as for one radius. Patches must be separated by at least the
larger radius: centre arclength >= eps_i + eps_j + max(eps_i, eps_j), so that
patch i lies in the far-field region (arclength > 2 eps_j) of every other
patch j.

Fields (Sections 2.2, 2.3 and eq. l2res with each patch's own radius):
potential integrates every patch by its own radius's radial rule and density
profiles (field._patch_quadrature with that radius's one-patch solve), a point
on patch i taking patch i's term from its data; l2_residual uses the rule of
field.residual_grid on [0, eps_i] and |Gamma_i| of eps_i.

Pins (tests/test_oracle_multitype.py): two types of equal radius reproduce
the single-radius system and the single-radius field; the compressed operator
equals the uncompressed one (each patch's own fine grid and densities); the
solved densities meet the absorbing condition on every patch of both radii,
by the on-surface sums and by the field; the interior field's normal
derivative on the reflecting surface is -I_sigma; a single patch of each type
gives its own one-patch scalars.
"""
from __future__ import annotations

import math

import numpy as np

from . import field, zernike
from .greens import INTERIOR, g_offsurface
from .system import frames, green_block, patch_points, rhs


class Layout:
    def __init__(self, centers, types, tabs):
        self.c = np.asarray(centers, dtype=np.float64)
        self.types = np.asarray(types, dtype=np.int64)
        self.tabs = list(tabs)
        self.N = len(self.c)
        self.e1, self.e2 = frames(self.c)
        self.problem = self.tabs[0].problem
        self.K = self.tabs[0].K
        self.Z = [patch_points(self.c[i:i + 1], self.e1[i:i + 1], self.e2[i:i + 1],
                               self.tabs[self.types[i]].node_t, self.tabs[self.types[i]].node_theta)[0]
                  for i in range(self.N)]
        self.S = [patch_points(self.c[i:i + 1], self.e1[i:i + 1], self.e2[i:i + 1],
                               self.tabs[self.types[i]].skel_t, self.tabs[self.types[i]].skel_theta)[0]
                  for i in range(self.N)]

    def tab(self, i):
        return self.tabs[self.types[i]]


def incoming_dense(lay: Layout, x):
    U = np.zeros((lay.N, len(lay.Z[0])))
    rho = [x[j] @ lay.tab(j).T.T for j in range(lay.N)]
    for i in range(lay.N):
        for j in range(lay.N):
            if j != i:
                U[i] += green_block(lay.Z[i], lay.S[j], lay.problem) @ rho[j]
    return U


def matvec_dense(lay: Layout, x):
    P = lay.tabs[0].P
    return x + incoming_dense(lay, x) @ P.T


def dense_matrix(lay: Layout):
    K, N, P = lay.K, lay.N, lay.tabs[0].P
    A = np.eye(K * N)
    for i in range(N):
        for j in range(N):
            if j != i:
                A[i * K:(i + 1) * K, j * K:(j + 1) * K] = P @ green_block(lay.Z[i], lay.S[j], lay.problem) @ lay.tab(j).T
    return A


def scalars(lay: Layout, x):
    flux = np.array([x[i] @ lay.tab(i).I for i in range(lay.N)])
    Is = float(np.sum(flux))
    out = {"I_sigma": Is, "flux": flux}
    if lay.problem == INTERIOR:
        out["mu"] = 1.0 / (3.0 * Is) - 0.6
    else:
        out["J_paper"] = -Is
        out["capture_rate"] = 4.0 * math.pi * Is
    return out


def solve_dense(lay: Layout):
    A = dense_matrix(lay)
    x = np.linalg.solve(A, rhs(lay.N, lay.K).ravel()).reshape(lay.N, lay.K)
    out = scalars(lay, x)
    out["x"] = x
    return out


def matvec_uncompressed(lay: Layout, ops, x):
    """y_i = x_i + P sum_{j != i} S_ij B_{tau_j} x_j with each patch's own fine
    grid (ops: the OnePatch of each type)."""
    P = lay.tabs[0].P
    Xf, sw = [], []
    for j in range(lay.N):
        op = ops[lay.types[j]]
        Xf.append(patch_points(lay.c[j:j + 1], lay.e1[j:j + 1], lay.e2[j:j + 1], op.fine_t, op.fine_theta)[0])
        sw.append((op.B @ x[j]) * op.w)
    y = x.copy()
    for i in range(lay.N):
        u = np.zeros(len(lay.Z[i]))
        for j in range(lay.N):
            if j != i:
                u += green_block(lay.Z[i], Xf[j], lay.problem) @ sw[j]
        y[i] += P @ u
    return y


def patch_residual(lay: Layout, ops, x, i, t, theta):
    """v - 1 at points (t, theta) of patch i: patch i's own term from its data
    sum_k x_ik Z_k(t/eps_i, theta), every other patch by its fine quadrature."""
    tab = lay.tab(i)
    self_part = np.zeros(len(t))
    for k, (n, m) in enumerate(zernike.modes(tab.M)):
        self_part += x[i, k] * zernike.basis(n, m, t / tab.eps, theta)
    X = patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], t, theta)[0]
    far = np.zeros(len(t))
    for j in range(lay.N):
        if j != i:
            op = ops[lay.types[j]]
            Xf = patch_points(lay.c[j:j + 1], lay.e1[j:j + 1], lay.e2[j:j + 1], op.fine_t, op.fine_theta)[0]
            far += green_block(X, Xf, lay.problem) @ ((op.B @ x[j]) * op.w)
    return self_part + far - 1.0


def on_patch(lay: Layout, point, tol: float = 1e-12):
    """Index of the patch containing `point` (on the sphere), or -1."""
    p = np.asarray(point, dtype=np.float64)
    if abs(np.linalg.norm(p) - 1.0) > tol:
        return -1
    ang = np.arctan2(np.linalg.norm(np.cross(lay.c, p), axis=1), lay.c @ p)
    i = int(np.argmin(ang))
    return i if ang[i] <= lay.tab(i).eps * (1 + tol) else -1


def self_term(lay: Layout, x, i, point):
    """sum_k x_ik Z_k(t/eps_i, theta) at a point of patch i."""
    p = np.asarray(point, dtype=np.float64)
    tab = lay.tab(i)
    t = math.atan2(np.linalg.norm(np.cross(lay.c[i], p)), float(lay.c[i] @ p))
    th = math.atan2(float(lay.e2[i] @ p), float(lay.e1[i] @ p))
    r = min(t / tab.eps, 1.0)
    return sum(x[i, k] * float(zernike.basis(n, m, r, th)) for k, (n, m) in enumerate(zernike.modes(tab.M)))


def potential(lay: Layout, ops, x, points, ntheta: int = 256):
    """u (exterior) or v (interior) at each of `points` (n, 3); ops: the
    OnePatch of each type."""
    points = np.atleast_2d(np.asarray(points, dtype=np.float64))
    quad = [field._patch_quadrature(lay, ops[lay.types[j]], x, j, ntheta) for j in range(lay.N)]
    out = np.zeros(len(points))
    for a, p in enumerate(points):
        i = on_patch(lay, p)
        for j in range(lay.N):
            if j == i:
                out[a] += self_term(lay, x, i, p)
            else:
                pts, sw = quad[j]
                out[a] += float(np.sum(g_offsurface(p[None, :], pts, lay.problem) * sw))
    return out


def l2_residual(lay: Layout, ops, x, i: int, nt: int = 20, ntheta: int = 40, ntheta_quad: int = 256):
    """(1/|Gamma_i|) ||v - 1||_{L2(Gamma_i)} on patch i (eq. l2res) with eps_i."""
    eps = lay.tab(i).eps
    t, th, w = field.residual_grid(eps, nt, ntheta)
    pts = patch_points(lay.c[i:i + 1], lay.e1[i:i + 1], lay.e2[i:i + 1], t, th)[0]
    r = potential(lay, ops, x, pts, ntheta_quad) - 1.0
    area = 2.0 * math.pi * (1.0 - math.cos(eps))
    return math.sqrt(float(np.sum(w * r * r))) / area, r
