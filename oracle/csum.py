"""ctypes wrapper of the oracle's plain C all-pairs Green's sum (csum.c).

TEST INFRASTRUCTURE (oracle). The shared object is built by
`build_csum()` with gcc (called from the repository's build step, or on
first use).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "csum.c"
_SO = _HERE / "_csum.so"
_lib = None


def build_csum(force: bool = False) -> Path:
    if force or not _SO.exists() or _SO.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _SO.with_suffix(".so.tmp")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", str(_SRC),
                               "-o", str(tmp), "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build_csum()
        lib = ctypes.CDLL(str(_SO))
        lib.nce_oracle_incoming.restype = None
        lib.nce_oracle_incoming.argtypes = [
            ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_void_p, ctypes.c_long,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_long, ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


def incoming(problem: int, Z: np.ndarray, S: np.ndarray, rho: np.ndarray, targets) -> np.ndarray:
    """U[a, k] = sum_{j != targets[a]} sum_m G(|Z[targets[a], k] - S[j, m]|) rho[j, m]."""
    lib = _load()
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    tg = np.ascontiguousarray(np.asarray(targets, dtype=np.int64))
    N, nz, _ = Z.shape
    ns = S.shape[1]
    U = np.empty((len(tg), nz))
    lib.nce_oracle_incoming(int(problem), N, nz, Z.ctypes.data, ns, S.ctypes.data,
                            rho.ctypes.data, len(tg), tg.ctypes.data, U.ctypes.data)
    return U


def incoming_layout(lay, x: np.ndarray, targets=None) -> np.ndarray:
    """Same as system.incoming_dense, via the C loop."""
    rho = x @ lay.tab.T.T
    tg = np.arange(lay.N) if targets is None else np.asarray(targets)
    return incoming(lay.tab.problem, lay.Z, lay.S, rho, tg)
