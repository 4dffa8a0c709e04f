"""Seeded synthetic patch layouts and random coefficient vectors.

This module is the only code shared by the CPU oracle and the GPU library's
tests and benchmark. It produces inputs only -- patch centres on the unit
sphere and random vectors -- and holds none of the solver's arithmetic.

The patch model is the paper's: N disk-shaped patches of common arclength
radius eps on the unit sphere, whose centres are at least 3*eps apart in
arclength (Section 3, "well-separated" assumption). Layouts follow the
shapes of the paper's experiments (Section 10.2): uniformly random
well-separated centres, Fibonacci spiral points, and clustered centres.

Every generator takes an integer seed and uses
numpy.random.Generator(PCG64(seed)), so both sides of a parity test see
bit-identical inputs.
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

__all__ = [
    "rng",
    "geodesic",
    "uniform_centers",
    "vmf_centers",
    "fibonacci_centers",
    "min_separation",
    "random_coeffs",
    "eps_from_area_fraction",
    "multi_radius_centers",
    "CONFIGS",
    "config_layout",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def geodesic(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Arclength between unit vectors (rows), atan2 form (accurate at all angles)."""
    cr = np.cross(a, b)
    return np.arctan2(np.linalg.norm(cr, axis=-1), np.sum(a * b, axis=-1))


class _CellHash:
    """3-D uniform grid over [-1,1]^3 used to find already-accepted centres
    that could lie within arclength `sep` of a candidate."""

    def __init__(self, sep: float):
        # chord length corresponding to arclength sep; points closer than
        # `sep` in arclength are closer than `h` in chord distance.
        self.h = 2.0 * math.sin(min(sep, math.pi) / 2.0) * (1.0 + 1e-12)
        self.h = max(self.h, 1e-12)
        self.cells: Dict[Tuple[int, int, int], List[int]] = {}

    def key(self, p: np.ndarray) -> Tuple[int, int, int]:
        return (int(math.floor(p[0] / self.h)), int(math.floor(p[1] / self.h)),
                int(math.floor(p[2] / self.h)))

    def near(self, p: np.ndarray):
        kx, ky, kz = self.key(p)
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    lst = self.cells.get((kx + dx, ky + dy, kz + dz))
                    if lst:
                        yield from lst

    def add(self, p: np.ndarray, idx: int) -> None:
        self.cells.setdefault(self.key(p), []).append(idx)


def _accept_loop(N: int, eps: float, propose, max_attempts: int, sep_factor: float = 3.0
                 ) -> np.ndarray:
    sep = sep_factor * eps * (1.0 + 1e-9)  # strict margin over the 3*eps rule
    grid = _CellHash(sep)
    out = np.empty((N, 3))
    n = 0
    attempts = 0
    while n < N:
        batch = propose(min(4096, max(64, 2 * (N - n))))
        for p in batch:
            attempts += 1
            if attempts > max_attempts:
                raise RuntimeError(
                    f"layout generator: could only place {n} of {N} patches "
                    f"(eps={eps}) within {max_attempts} attempts")
            ok = True
            for j in grid.near(p):
                q = out[j]
                ang = math.atan2(np.linalg.norm(np.cross(p, q)), float(p @ q))
                if ang < sep:
                    ok = False
                    break
            if ok:
                out[n] = p
                grid.add(p, n)
                n += 1
                if n == N:
                    break
    return out


def multi_radius_centers(N: int, radii, seed: int, weights=None):
    """Uniform random centres carrying one of several patch radii each (a
    type index into `radii`, drawn with probabilities `weights`, uniform by
    default); any two patches i, j are accepted only with centre arclength >=
    eps_i + eps_j + max(eps_i, eps_j), the gap between them at least the larger
    radius (3 eps for equal radii). Returns (centres N x 3, types N)."""
    radii = np.asarray(radii, dtype=np.float64)
    w = np.full(len(radii), 1.0 / len(radii)) if weights is None else np.asarray(weights, dtype=np.float64)
    g = rng(seed)
    grid = _CellHash(3.0 * float(radii.max()) * (1.0 + 1e-9))
    out = np.empty((N, 3))
    typ = np.empty(N, dtype=np.int64)
    n = attempts = 0
    while n < N:
        v = g.standard_normal(3)
        p = v / np.linalg.norm(v)
        t = int(g.choice(len(radii), p=w))
        attempts += 1
        if attempts > 1000 * N:
            raise RuntimeError(f"layout generator: could only place {n} of {N} patches")
        ok = True
        for j in grid.near(p):
            sep = radii[t] + radii[typ[j]] + max(radii[t], radii[typ[j]])
            if math.atan2(np.linalg.norm(np.cross(p, out[j])), float(p @ out[j])) < sep * (1.0 + 1e-9):
                ok = False
                break
        if ok:
            out[n] = p
            typ[n] = t
            grid.add(p, n)
            n += 1
    return out, typ


def uniform_centers(N: int, eps: float, seed: int) -> np.ndarray:
    """Uniform random centres with centre arclength >= 3*eps (rejection
    sampling; proposals are normalised standard-normal 3-vectors)."""
    g = rng(seed)

    def propose(m):
        v = g.standard_normal((m, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    return _accept_loop(N, eps, propose, 1000 * N)


def vmf_centers(N: int, eps: float, seed: int, kappa: float = 5.0) -> np.ndarray:
    """Clustered centres: proposals from a von Mises-Fisher distribution
    (concentration kappa) about a pole drawn uniformly from the same RNG,
    with the same 3*eps acceptance rule (a jammed cluster that spills
    outward when the vMF density is too high)."""
    g = rng(seed)
    pole = g.standard_normal(3)
    pole /= np.linalg.norm(pole)
    a = np.array([0.0, 0.0, 1.0]) if abs(pole[2]) < 0.9 else np.array([1.0, 0.0, 0.0])
    e1 = a - (a @ pole) * pole
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(pole, e1)

    def propose(m):
        u = g.random(m)
        w = 1.0 + np.log(u + (1.0 - u) * math.exp(-2.0 * kappa)) / kappa
        w = np.clip(w, -1.0, 1.0)
        phi = 2.0 * math.pi * g.random(m)
        s = np.sqrt(np.maximum(0.0, 1.0 - w * w))
        v = (w[:, None] * pole[None, :] + (s * np.cos(phi))[:, None] * e1[None, :]
             + (s * np.sin(phi))[:, None] * e2[None, :])
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    return _accept_loop(N, eps, propose, 1000 * N)


def fibonacci_centers(N: int, variant: str = "half") -> np.ndarray:
    """Fibonacci spiral points (deterministic, no seed).

    variant "half":   z_k = 1 - (2k+1)/N,        azimuth k * golden angle
    variant "ends":   z_k = 1 - 2k/(N-1),        azimuth k * golden angle
    """
    k = np.arange(N, dtype=np.float64)
    ga = math.pi * (3.0 - math.sqrt(5.0))
    if variant == "half":
        z = 1.0 - (2.0 * k + 1.0) / N
    elif variant == "ends":
        z = 1.0 - 2.0 * k / (N - 1) if N > 1 else np.array([1.0])
    else:
        raise ValueError(variant)
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = ga * k
    v = np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def min_separation(c: np.ndarray) -> float:
    """Smallest pairwise centre arclength (O(N^2); for small N)."""
    N = len(c)
    best = math.inf
    for i in range(N - 1):
        d = geodesic(np.broadcast_to(c[i], (N - 1 - i, 3)), c[i + 1:])
        best = min(best, float(d.min()))
    return best


def random_coeffs(N: int, K: int, seed: int, decay: float = 0.0) -> np.ndarray:
    """Random N x K coefficient matrix (row-major, patch-major) of standard
    normals, optionally scaled by exp(-decay * column) to mimic spectral decay."""
    x = rng(seed).standard_normal((N, K))
    if decay:
        x *= np.exp(-decay * np.arange(K))[None, :]
    return x


def eps_from_area_fraction(f: float, N: int) -> float:
    """Patch radius from the small-eps area fraction f = eps^2 N / 4 (Section 10)."""
    return 2.0 * math.sqrt(f / N)


# The five named workloads (problem: 0 interior / narrow escape, 1 exterior / narrow capture).
CONFIGS = {
    "cfg1": dict(problem=1, N=10, eps=0.1, layout="uniform", seed=1),
    "cfg2": dict(problem=0, N=1000, eps=0.01, layout="uniform", seed=2),
    "cfg3": dict(problem=1, N=10000, eps=0.005, layout="vmf", seed=3),
    "cfg5": dict(problem=0, N=100000, eps=0.001, layout="uniform", seed=5),
}


def batch_member(b: int) -> dict:
    """Member b (0..255) of the batched workload: interior if b even,
    eps = 0.01 if b mod 4 < 2 else 0.02; N ~ U{100..5000} at eps=0.01 and
    U{100..1500} at eps=0.02 (larger N does not fit at separation 3*eps)."""
    g = rng(4000 + b)
    eps = 0.01 if (b % 4) < 2 else 0.02
    hi = 5000 if eps == 0.01 else 1500
    N = int(g.integers(100, hi + 1))
    return dict(problem=0 if b % 2 == 0 else 1, N=N, eps=eps, layout="uniform", seed=4000 + b)


def config_layout(cfg: dict) -> np.ndarray:
    if cfg["layout"] == "uniform":
        return uniform_centers(cfg["N"], cfg["eps"], cfg["seed"])
    if cfg["layout"] == "vmf":
        return vmf_centers(cfg["N"], cfg["eps"], cfg["seed"])
    raise ValueError(cfg["layout"])
