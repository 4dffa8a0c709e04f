"""Host checks of the coarse-space deflation basis (library host code built
with g++, no GPU): orthonormal columns spanning the polynomials of degree <= 3
on the patch centres, equal to the modified Gram-Schmidt result written out
here in numpy."""
import os
import subprocess
from pathlib import Path

import numpy as np
import pytest

import layouts

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1906_04209_amd" / "csrc"


def harmonic_polys(c):
    """The 16 harmonic polynomials of degree <= 3 at the centres (N x 16)."""
    x, y, z = c[:, 0], c[:, 1], c[:, 2]
    r2 = x * x + y * y
    return np.stack([np.ones_like(x), x, y, z, x * y, y * z, z * x, x * x - y * y, 2 * z * z - r2,
                     x * (x * x - 3 * y * y), y * (3 * x * x - y * y), z * (x * x - y * y), x * y * z,
                     x * (4 * z * z - r2), y * (4 * z * z - r2), z * (2 * z * z - 3 * r2)], axis=1)


def mgs(A):
    Q = []
    for j in range(A.shape[1]):
        v = A[:, j].copy()
        n0 = np.linalg.norm(v)
        for _ in range(2):
            for q in Q:
                v -= (q @ v) * q
        if np.linalg.norm(v) > 1e-8 * n0:
            Q.append(v / np.linalg.norm(v))
    return np.stack(Q, axis=1)


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    out = tmp_path_factory.mktemp("defl") / "deflate_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", str(ROOT / "tests" / "host" / "deflate_check.cpp"),
                           str(CSRC / "deflate_basis.cpp"), "-o", str(out)])
    return out


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_deflation_basis(exe, tmp_path, kind):
    c = layouts.uniform_centers(400, 0.01, 51) if kind == "uniform" else layouts.vmf_centers(400, 0.01, 52)
    fr = np.zeros((len(c), 9))
    fr[:, :3] = c
    f = tmp_path / "in.txt"
    with open(f, "w") as fh:
        fh.write(f"{len(c)}\n")
        np.savetxt(fh, fr, fmt="%.17g")
    out = subprocess.run([str(exe), str(f)], capture_output=True, text=True, check=True).stdout.splitlines()
    # bit-identical whatever the thread count (fixed-order reductions)
    for nt in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=nt)
        assert subprocess.run([str(exe), str(f)], capture_output=True, text=True, check=True,
                              env=env).stdout.splitlines() == out
    k = int(out[0])
    Z = np.loadtxt(out[1:])
    assert k == 16
    assert np.max(np.abs(Z.T @ Z - np.eye(16))) < 1e-12
    # spans every polynomial of degree <= 3 on the centres (x^2 + y^2 + z^2 = 1 there)
    x, y, zz = c[:, 0], c[:, 1], c[:, 2]
    for p in (x ** 3, x * y * zz + 0.3 * zz ** 2, y ** 2 - 0.5, x * zz ** 2 + y ** 3):
        assert np.linalg.norm(p - Z @ (Z.T @ p)) < 1e-10 * np.linalg.norm(p)
    # the same columns as Gram-Schmidt on the harmonic polynomials in this order
    Q = mgs(harmonic_polys(c))
    assert np.max(np.abs(Z - Q)) < 1e-10


@pytest.fixture(scope="module")
def inv_exe(tmp_path_factory):
    out = tmp_path_factory.mktemp("inv") / "invert_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", str(ROOT / "tests" / "host" / "invert_check.cpp"),
                           str(CSRC / "deflate_basis.cpp"), "-o", str(out)])
    return out


def _invert(exe, tmp_path, T):
    f = tmp_path / "T.txt"
    with open(f, "w") as fh:
        fh.write(f"{len(T)}\n")
        np.savetxt(fh, T, fmt="%.17g")
    out = subprocess.run([str(exe), str(f)], capture_output=True, text=True, check=True).stdout.splitlines()
    return out[0], (np.loadtxt(out[1:]) if out[0] == "ok" else None)


@pytest.mark.parametrize("k", [16, 7, 1])
def test_deflation_inverse_matches_numpy(inv_exe, tmp_path, k):
    """M = T^-1 - I on the first k rows and columns, zero padding beyond, for a
    nonsymmetric T whose pivots need row exchanges (zero leading diagonal)."""
    g = np.random.Generator(np.random.PCG64(70 + k))
    T = np.eye(k) + 0.3 * g.standard_normal((k, k))
    if k > 1:
        T[0, 0] = 0.0
    status, M = _invert(inv_exe, tmp_path, T)
    assert status == "ok"
    ref = np.zeros((16, 16))
    ref[:k, :k] = np.linalg.inv(T) - np.eye(k)
    assert np.max(np.abs(M - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_deflation_inverse_singular(inv_exe, tmp_path):
    """A singular T is reported (the library then leaves the layout undeflated)."""
    T = np.eye(5)
    T[3] = T[1]
    status, _ = _invert(inv_exe, tmp_path, T)
    assert status == "singular"
