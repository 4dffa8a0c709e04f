"""Per-(problem, eps, M, tol_id) precompute driver for the oracle (paper Section 8, Step 1).

TEST INFRASTRUCTURE (oracle).

Step 1(a) one-patch solve S B = Q -> B, w (onepatch), 1(b) T = Pi W B by
ID (idcomp), 1(c) I = w^T B. The outputs (T, skeleton coordinates, I) are
cached as .npz: first under tests/golden/tables (committed, written by
tests/golden/make_golden.py which calls only this package), then in a local
cache directory ($NCE_ORACLE_CACHE, default oracle/_cache, not committed).
"""
from __future__ import annotations

import hashlib
import os
from pathlib import Path

import numpy as np

from . import idcomp, onepatch, zernike
from .system import Tables

_ROOT = Path(__file__).resolve().parent.parent
GOLDEN_DIR = _ROOT / "tests" / "golden" / "tables"


def _cache_dir() -> Path:
    return Path(os.environ.get("NCE_ORACLE_CACHE", str(_ROOT / "oracle" / "_cache")))


def key(problem: int, eps: float, M: int, tol_id: float, ntheta: int = onepatch.NTHETA_F) -> str:
    return f"p{problem}_eps{eps:.10g}_M{M}_id{tol_id:.0e}_nt{ntheta}"


def _assemble(problem, eps, M, T, st, sth, I) -> Tables:
    P = zernike.transform(M)
    R, TH = zernike.node_polar(M)
    return Tables(problem, eps, M, T, st, sth, I, P, eps * R, TH)


def compute(problem: int, eps: float, M: int = 15, tol_id: float = 1e-12,
            ntheta: int = onepatch.NTHETA_F):
    """Full precompute; returns (Tables, OnePatch, Compressed)."""
    op = onepatch.solve_one_patch(eps, problem, M=M, ntheta=ntheta)
    cp = idcomp.interpolative_decomposition(op, tol_id)
    tab = _assemble(problem, eps, M, cp.T, cp.skel_t, cp.skel_theta, op.I)
    return tab, op, cp


def save(tab: Tables, path: Path) -> str:
    path.parent.mkdir(parents=True, exist_ok=True)
    np.savez(path, T=tab.T, skel_t=tab.skel_t, skel_theta=tab.skel_theta, I=tab.I,
             meta=np.array([tab.problem, tab.eps, tab.M], dtype=np.float64))
    return hashlib.sha256(path.read_bytes()).hexdigest()


def load(path: Path) -> Tables:
    z = np.load(path, allow_pickle=False)
    prob, eps, M = z["meta"]
    return _assemble(int(prob), float(eps), int(M), z["T"], z["skel_t"], z["skel_theta"], z["I"])


def get(problem: int, eps: float, M: int = 15, tol_id: float = 1e-12,
        ntheta: int = onepatch.NTHETA_F) -> Tables:
    k = key(problem, eps, M, tol_id, ntheta)
    for d in (GOLDEN_DIR, _cache_dir()):
        f = d / (k + ".npz")
        if f.exists():
            return load(f)
    tab, _, _ = compute(problem, eps, M, tol_id, ntheta)
    save(tab, _cache_dir() / (k + ".npz"))
    return tab
