"""The C-ABI library loads, exports every declared symbol, and rejects bad
input before touching the GPU (host-side validation only; no compute calls)."""
import ctypes
import re
from pathlib import Path

import numpy as np
import pytest

import paper_1906_04209_amd as nce

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    txt = (ROOT / "include" / "nce.h").read_text()
    return sorted(set(re.findall(r"\b(nce_[a-z0-9_]+)\s*\(", txt)))


def test_header_matches_binding_list():
    assert _declared() == sorted(nce.SYMBOLS)


def test_library_exports_every_symbol():
    lib = nce.load()
    for s in _declared():
        assert hasattr(lib, s), s


def _setup(centers, eps, **kw):
    lib = nce.load()
    o = nce.Opts()
    lib.nce_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    h = ctypes.c_void_p()
    c = np.ascontiguousarray(centers, dtype=np.float64)
    rc = lib.nce_setup(c.ctypes.data, len(c), eps, ctypes.byref(o), ctypes.byref(h))
    return rc, lib.nce_last_error().decode(), h


def test_default_opts():
    lib = nce.load()
    o = nce.Opts()
    lib.nce_default_opts(ctypes.byref(o))
    assert (o.M, o.tol_id, o.tol_grid, o.tol_gmres, o.precision) == (15, 1e-11, 1e-8, 1e-10, 0)
    assert (o.tol_grid_fp32, o.tol_id_fp32, o.tol_coarse, o.deflation) == (3e-4, 1e-5, 1e-5, 1)


@pytest.mark.parametrize("case", ["empty", "nonunit", "nan", "eps0", "epsbig", "badM", "bigM", "badprob",
                                  "badcoarse", "badgrid32", "baddefl"])
def test_invalid_arguments(case):
    c = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    eps, kw = 0.1, {}
    if case == "empty":
        c = np.zeros((0, 3))
    elif case == "nonunit":
        c = c * 1.001
    elif case == "nan":
        c[1, 0] = np.nan
    elif case == "eps0":
        eps = 0.0
    elif case == "epsbig":
        eps = 1.2
    elif case == "badM":
        kw = {"M": -1}
    elif case == "bigM":
        kw = {"M": 16}   # 2 (M+1)^2 = 578 sampling nodes: more than the kernels hold
    elif case == "badprob":
        kw = {"problem": 3}
    elif case == "badcoarse":
        kw = {"tol_coarse": 0.5}
    elif case == "badgrid32":
        kw = {"tol_grid_fp32": 0.5}
    elif case == "baddefl":
        kw = {"deflation": 2}
    rc, msg, h = _setup(c, eps, **kw)
    assert rc == -1 and not h.value and msg


def test_null_handles_rejected():
    """Entry points on a NULL context or batch, and a batch of no
    configurations, fail with NCE_EINVAL and a message, before any device
    work."""
    lib = nce.load()
    h = ctypes.c_void_p()
    mu = ctypes.c_double()
    for fn, args in [(lib.nce_set_deflation, (None, 1)), (lib.nce_batch_set_deflation, (None, 1)),
                     (lib.nce_batch_set_warm_start, (None, None, 1)), (lib.nce_matvec, (None, None, None, 0)),
                     (lib.nce_solve_interior, (None, None, None, ctypes.byref(mu), None)),
                     (lib.nce_solve_batch, (None, None, None, None)), (lib.nce_batch_matvec, (None, None, None, 0)),
                     (lib.nce_setup_batch, (None, None, None, None, 0, None, ctypes.byref(h))),
                     (lib.nce_mlp_forward_noalloc, (None, None, 1, None, None))]:
        assert fn(*args) == -1, fn.__name__
        assert lib.nce_last_error()
    assert not h.value


def test_separation_rule():
    # centres 2.9 eps apart in arclength violate the 3 eps rule (Section 3)
    eps = 0.05
    a = 2.9 * eps
    c = np.array([[0.0, 0.0, 1.0], [np.sin(a), 0.0, np.cos(a)]])
    rc, msg, h = _setup(c, eps)
    assert rc == -2 and "closer than 3 eps" in msg


def test_strerror_codes():
    lib = nce.load()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        assert lib.nce_strerror(code)


def test_radii_validation():
    """nce_setup_radii rejects bad radii, more than 8 of them and patches
    closer than eps_i + eps_j + max(eps_i, eps_j), before any device work."""
    lib = nce.load()
    o = nce.Opts()
    lib.nce_default_opts(ctypes.byref(o))
    h = ctypes.c_void_p()
    c = np.array([[0.0, 0.0, 1.0], [np.sin(0.35), 0.0, np.cos(0.35)]])
    for r, want in (([0.1, -0.1], -1), ([0.1, 1.2], -1), ([0.1, 0.15], -2)):
        rr = np.ascontiguousarray(r, dtype=np.float64)
        assert lib.nce_setup_radii(c.ctypes.data, rr.ctypes.data, 2, ctypes.byref(o), ctypes.byref(h)) == want
        assert lib.nce_last_error() and not h.value
    # 0.1 + 0.15 + 0.15 = 0.4 > 0.35 failed above; 0.1 + 0.12 + 0.12 = 0.34 passes the separation test
    cc = np.array([[np.cos(2 * np.pi * k / 9), np.sin(2 * np.pi * k / 9), 0.0] for k in range(9)])
    rr = np.linspace(0.01, 0.02, 9)
    assert lib.nce_setup_radii(cc.ctypes.data, rr.ctypes.data, 9, ctypes.byref(o), ctypes.byref(h)) == -1
    assert b"8" in lib.nce_last_error()
