"""Host (CPU) checks of the library's cube-sphere tree construction: every
ordered pair of patches is summed exactly once (near list or one interaction
list on the target's ancestor path, as in Section 8 Step 3's note), every
incoming grid covers its members and lies in its sources' far-field regions."""
import os
import subprocess
from pathlib import Path

import numpy as np
import pytest

import layouts

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_1906_04209_amd" / "csrc"


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("tree")
    out = d / "tree_check"
    # with OpenMP, as the library builds it: the boxes of a level are processed in parallel
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-I", str(CSRC),
                           str(ROOT / "tests" / "host" / "tree_check.cpp"), str(CSRC / "tree_build.cpp"), "-o", str(out)])
    return out


def _run(exe, tmp_path, c, eps, tol=1e-8, threads=None):
    f = tmp_path / "c.txt"
    with open(f, "w") as fh:
        fh.write(f"{len(c)}\n")
        np.savetxt(fh, c, fmt="%.17g")
    env = dict(os.environ)
    if threads is not None:
        env["OMP_NUM_THREADS"] = str(threads)
    r = subprocess.run([str(exe), str(f), repr(eps), repr(tol)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK"), r.stdout
    return r.stdout


@pytest.mark.parametrize("N,eps,seed", [(2, 0.1, 1), (10, 0.1, 1), (300, 0.02, 3), (2000, 0.005, 4)])
def test_uniform_coverage(exe, tmp_path, N, eps, seed):
    out = _run(exe, tmp_path, layouts.uniform_centers(N, eps, seed), eps)
    print(out)
    if N >= 2000:
        # the far-source grids are exercised (boxes with a second, coarser grid)
        assert int(out.split("split ")[1].split()[0]) > 0


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_build_independent_of_thread_count(exe, tmp_path, kind):
    """The parallel build (boxes of a level over OpenMP threads, grids numbered
    afterwards in box order) gives the same tree, byte for byte, on one thread
    and on eight."""
    eps = 0.005
    c = layouts.uniform_centers(2000, eps, 4) if kind == "uniform" else layouts.vmf_centers(1500, eps, 9)
    hashes = {n: _run(exe, tmp_path, c, eps, threads=n).split("hash ")[1].split()[0] for n in (1, 8)}
    assert hashes[1] == hashes[8], hashes


def test_clustered_coverage(exe, tmp_path):
    print(_run(exe, tmp_path, layouts.vmf_centers(1500, 0.005, 9), 0.005))


def test_cube_corner_and_edges(exe, tmp_path):
    # centres on cube edges and corners exercise the wrap-around neighbours
    v = []
    for s in [(1, 1, 1), (1, 1, -1), (1, -1, 1), (-1, 1, 1), (1, 0, 1), (0, 1, 1), (1, 1, 0), (-1, -1, -1)]:
        x = np.array(s, float)
        v.append(x / np.linalg.norm(x))
    c = np.vstack([v, layouts.uniform_centers(200, 0.01, 12)])
    keep = [0]
    for i in range(1, len(c)):
        if all(np.arccos(np.clip(c[i] @ c[k], -1, 1)) >= 0.031 for k in keep):
            keep.append(i)
    print(_run(exe, tmp_path, c[keep], 0.01))


@pytest.fixture(scope="module")
def forest_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("forest")
    out = d / "forest_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-I", str(CSRC), str(ROOT / "tests" / "host" / "forest_check.cpp"),
                           str(CSRC / "tree_build.cpp"), "-o", str(out)])
    return out


def test_forest_coverage(forest_exe, tmp_path):
    """Several configurations in one numbering (trees and direct lists, one of a
    single patch): pairs only within a configuration, each exactly once."""
    eps = 0.02
    cfgs = [layouts.uniform_centers(n, eps, 70 + k) for k, n in enumerate([150, 1, 60, 400, 2, 33, 250])]
    f = tmp_path / "forest.txt"
    with open(f, "w") as fh:
        fh.write(f"{len(cfgs)}\n")
        for c in cfgs:
            fh.write(f"{len(c)}\n")
            np.savetxt(fh, c, fmt="%.17g")
    r = subprocess.run([str(forest_exe), str(f), repr(eps), "1e-8"], capture_output=True, text=True)
    print(r.stdout)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr


@pytest.fixture(scope="module")
def features_exe(tmp_path_factory):
    d = tmp_path_factory.mktemp("features")
    out = d / "features_check"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", str(ROOT / "tests" / "host" / "features_check.cpp"),
                           str(CSRC / "features.cpp"), "-o", str(out)])
    return out


def _frames(c):
    """Orthonormal tangent frames (c, e1, e2) per centre."""
    a = np.where(np.abs(c[:, 2:3]) > 1 / np.sqrt(2), [[1.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]])
    e1 = a - np.sum(a * c, axis=1, keepdims=True) * c
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(c, e1)
    return np.concatenate([c, e1, e2], axis=1)


def _features_brute(fr, eps, problem, a):
    """The feature definition written out by brute force over all pairs."""
    N = len(fr)
    c = fr[:, :3]
    cr = np.linalg.norm(np.cross(c[:, None, :], c[None, :, :]), axis=-1)
    geo = np.arctan2(cr, c @ c.T)
    np.fill_diagonal(geo, np.inf)
    out = np.zeros((N, 56))
    area = N * np.sin(0.5 * eps) ** 2
    for i in range(N):
        nb = np.argsort(geo[i], kind="stable")[:16]
        d = c[nb] - c[i]
        out[i, 0:48:3] = (d @ fr[i, 3:6]) / eps / 16.0
        out[i, 1:48:3] = (d @ fr[i, 6:9]) / eps / 16.0
        out[i, 2:48:3] = 4.0 / (geo[i, nb] / eps)
        out[i, 48] = problem
        out[i, 49] = 10.0 * area
        for q, R in enumerate((8 * eps, 16 * eps, 32 * eps, 64 * eps)):
            R = min(R, np.pi)
            out[i, 50 + q] = np.sum(geo[i] <= R) / max((N - 1) * 0.5 * (1 - np.cos(R)), 1e-12)
        out[i, 54] = 10.0 * (a[i] / a.mean() - 1.0)
        out[i, 55] = a.mean()
    return out


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_features_match_brute_force(features_exe, tmp_path, kind):
    """Grid-accelerated neighbour features equal the all-pairs definition."""
    eps, prob = 0.01, 1
    if kind == "uniform":
        c = layouts.uniform_centers(500, eps, 31)
    else:
        c = layouts.vmf_centers(500, eps, 32)
    fr = _frames(c)
    a = 1.0 + 0.1 * np.random.default_rng(5).standard_normal(len(c))
    f = tmp_path / "in.txt"
    with open(f, "w") as fh:
        fh.write(f"{len(c)} {eps!r} {prob}\n")
        np.savetxt(fh, fr, fmt="%.17g")
        np.savetxt(fh, a, fmt="%.17g")
    r = subprocess.run([str(features_exe), str(f)], capture_output=True, text=True, check=True)
    got = np.loadtxt(r.stdout.splitlines())
    ref = _features_brute(fr, eps, prob, a)
    err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    print(f"{kind}: N={len(c)} max rel err {err.max():.2e}")
    assert err.max() < 1e-5
