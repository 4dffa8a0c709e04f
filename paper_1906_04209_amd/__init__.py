"""MI355X narrow capture / narrow escape solver (Kaye & Greengard), Python binding.

A thin ctypes layer over libnce.so (include/nce.h): it marshals arguments and
nothing else. Every step of the matrix-vector product and of the solves runs
in the library's HIP kernels; PyTorch provides device memory and the stream.
Importing works without a GPU; creating a context needs the built library and
a HIP device, and raises if either is missing (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
import os
from pathlib import Path
from typing import Optional

import numpy as np

__all__ = ["load", "Context", "Batch", "Mlp", "NCEError", "FEATURES", "INTERIOR", "EXTERIOR", "FP64", "MIXED",
           "FAR_AUTO", "FAR_DIRECT", "FAR_TREE", "LIB_PATH", "SYMBOLS"]

LIB_PATH = Path(__file__).resolve().parent / "libnce.so"

INTERIOR, EXTERIOR = 0, 1
FP64, MIXED = 0, 1
FAR_AUTO, FAR_DIRECT, FAR_TREE = 0, 1, 2

# every symbol include/nce.h declares
SYMBOLS = ["nce_default_opts", "nce_setup", "nce_destroy", "nce_dims", "nce_frames", "nce_work",
           "nce_matvec", "nce_matvec_profile", "nce_set_solver", "nce_solve_interior", "nce_solve_exterior", "nce_integral_vector",
           "nce_field", "nce_patch_residual", "nce_setup_radii", "nce_types", "nce_set_shapes",
           "nce_strerror", "nce_last_error", "nce_mlp_create", "nce_mlp_destroy", "nce_mlp_num_params",
           "nce_mlp_get_params", "nce_mlp_set_params", "nce_mlp_forward", "nce_mlp_forward_noalloc", "nce_mlp_loss_grad",
           "nce_mlp_train_step", "nce_features", "nce_set_warm_start", "nce_setup_batch",
           "nce_destroy_batch", "nce_batch_dims", "nce_batch_offsets", "nce_batch_work", "nce_batch_matvec",
           "nce_batch_set_solver", "nce_solve_batch", "nce_autotune", "nce_batch_autotune", "nce_coarse_solve",
           "nce_batch_set_warm_start", "nce_deflation_matrix", "nce_set_deflation", "nce_batch_set_deflation"]
FEATURES = 56


class Opts(ctypes.Structure):
    _fields_ = [("problem", ctypes.c_int), ("M", ctypes.c_int), ("tol_id", ctypes.c_double),
                ("tol_grid", ctypes.c_double), ("tol_gmres", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("precision", ctypes.c_int),
                ("far_field", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("cache_dir", ctypes.c_char_p), ("tol_grid_fp32", ctypes.c_double),
                ("tol_id_fp32", ctypes.c_double), ("tol_coarse", ctypes.c_double), ("deflation", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("iters_fp64", ctypes.c_int), ("iters_fp32", ctypes.c_int), ("outer", ctypes.c_int),
                ("used_fallback", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("t_solve_s", ctypes.c_double), ("rel_residual_x0", ctypes.c_double)]

    def asdict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NCEError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nce error {code}: {msg}")
        self.code = code


_lib = None


def load(path: Optional[os.PathLike] = None):
    """Load libnce.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(f"{p} is missing: build it with paper_1906_04209_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(str(p))
    vp, i64, dp, ip = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    lib.nce_default_opts.argtypes = [ctypes.POINTER(Opts)]
    lib.nce_default_opts.restype = None
    lib.nce_setup.argtypes = [vp, i64, ctypes.c_double, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    lib.nce_destroy.argtypes = [vp]
    lib.nce_destroy.restype = None
    lib.nce_dims.argtypes = [vp, ip, ip, ip, ip]
    lib.nce_frames.argtypes = [vp, vp]
    lib.nce_work.argtypes = [vp, ctypes.c_int, dp, dp, dp]
    lib.nce_matvec.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nce_matvec_profile.argtypes = [vp, vp, vp, ctypes.c_int, vp]
    lib.nce_set_solver.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.nce_solve_interior.argtypes = [vp, vp, vp, dp, ctypes.POINTER(Info)]
    lib.nce_solve_exterior.argtypes = [vp, vp, vp, dp, dp, ctypes.POINTER(Info)]
    lib.nce_integral_vector.argtypes = [vp, vp]
    lib.nce_set_shapes.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.nce_set_shapes.restype = ctypes.c_int
    lib.nce_setup_radii.argtypes = [vp, vp, i64, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    lib.nce_setup_radii.restype = ctypes.c_int
    lib.nce_types.argtypes = [vp, ip, vp, vp, vp]
    lib.nce_types.restype = ctypes.c_int
    lib.nce_field.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp]
    lib.nce_field.restype = ctypes.c_int
    lib.nce_patch_residual.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    lib.nce_patch_residual.restype = ctypes.c_int
    lib.nce_mlp_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                   ctypes.POINTER(vp)]
    lib.nce_mlp_destroy.argtypes = [vp]
    lib.nce_mlp_destroy.restype = None
    lib.nce_mlp_num_params.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
    lib.nce_mlp_get_params.argtypes = [vp, vp]
    lib.nce_mlp_set_params.argtypes = [vp, vp]
    lib.nce_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    lib.nce_mlp_forward_noalloc.argtypes = [vp, vp, i64, vp, vp]
    lib.nce_mlp_loss_grad.argtypes = [vp, vp, vp, i64, dp, vp, vp]
    lib.nce_mlp_train_step.argtypes = [vp, vp, vp, i64, ctypes.c_float, dp, vp]
    lib.nce_features.argtypes = [vp, vp]
    lib.nce_set_warm_start.argtypes = [vp, vp, ctypes.c_int]
    lib.nce_coarse_solve.argtypes = [vp, vp, ip, dp]
    lib.nce_coarse_solve.restype = ctypes.c_int
    lib.nce_deflation_matrix.argtypes = [vp, ip, dp]
    lib.nce_deflation_matrix.restype = ctypes.c_int
    lib.nce_set_deflation.argtypes = [vp, ctypes.c_int]
    lib.nce_set_deflation.restype = ctypes.c_int
    lib.nce_batch_set_deflation.argtypes = [vp, ctypes.c_int]
    lib.nce_batch_set_deflation.restype = ctypes.c_int
    for name in ("nce_mlp_create", "nce_mlp_num_params", "nce_mlp_get_params", "nce_mlp_set_params",
                 "nce_mlp_forward", "nce_mlp_forward_noalloc", "nce_mlp_loss_grad", "nce_mlp_train_step",
                 "nce_features",
                 "nce_set_warm_start"):
        getattr(lib, name).restype = ctypes.c_int
    lib.nce_setup_batch.argtypes = [vp, vp, vp, vp, ctypes.c_int, ctypes.POINTER(Opts), ctypes.POINTER(vp)]
    lib.nce_destroy_batch.argtypes = [vp]
    lib.nce_destroy_batch.restype = None
    lib.nce_batch_dims.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ip, ip]
    lib.nce_batch_offsets.argtypes = [vp, vp, vp]
    lib.nce_batch_work.argtypes = [vp, ctypes.c_int, dp, dp, dp]
    lib.nce_batch_matvec.argtypes = [vp, vp, vp, ctypes.c_int]
    lib.nce_batch_set_solver.argtypes = [vp, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.nce_solve_batch.argtypes = [vp, vp, vp, vp]
    lib.nce_autotune.argtypes = [vp, ctypes.c_int, vp]
    lib.nce_batch_autotune.argtypes = [vp, ctypes.c_int, vp]
    lib.nce_batch_set_warm_start.argtypes = [vp, vp, ctypes.c_int]
    lib.nce_batch_set_warm_start.restype = ctypes.c_int
    for name in ("nce_setup_batch", "nce_batch_dims", "nce_batch_offsets", "nce_batch_work", "nce_batch_matvec",
                 "nce_batch_set_solver", "nce_solve_batch", "nce_autotune", "nce_batch_autotune"):
        getattr(lib, name).restype = ctypes.c_int
    lib.nce_strerror.argtypes = [ctypes.c_int]
    lib.nce_strerror.restype = ctypes.c_char_p
    lib.nce_last_error.argtypes = []
    lib.nce_last_error.restype = ctypes.c_char_p
    for name in ("nce_setup", "nce_dims", "nce_frames", "nce_work", "nce_matvec", "nce_matvec_profile", "nce_set_solver", "nce_solve_interior",
                 "nce_solve_exterior", "nce_integral_vector"):
        getattr(lib, name).restype = ctypes.c_int
    if path is None:
        _lib = lib
    return lib


def _check(lib, rc: int, allow_notconv: bool = False) -> int:
    if rc == 0 or (allow_notconv and rc == 1):
        return rc
    raise NCEError(rc, lib.nce_last_error().decode() or lib.nce_strerror(rc).decode())


def _ptr(t, dtype=None) -> int:
    if t is None:
        return None
    import torch
    dt = dtype or torch.float64
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dt and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dt} CUDA tensor")
    return t.data_ptr()


class Mlp:
    """The warm-start network (nce_mlp_*): FP32 parameters and kernels on the GPU."""

    def __init__(self, n_in: int = FEATURES, width: int = 256, hidden: int = 3, n_out: int = 136, seed: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the network runs only on the GPU")
        self.lib = load()
        self.torch = torch
        self.shape = (n_in, width, hidden, n_out)
        h = ctypes.c_void_p()
        _check(self.lib, self.lib.nce_mlp_create(n_in, width, hidden, n_out, seed, ctypes.byref(h)))
        self.h = h
        n = ctypes.c_int64()
        _check(self.lib, self.lib.nce_mlp_num_params(h, ctypes.byref(n)))
        self.nparam = n.value
        self.stream = torch.cuda.Stream()

    def close(self):
        if getattr(self, "h", None):
            self.lib.nce_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.empty(self.nparam, dtype=np.float32)
        _check(self.lib, self.lib.nce_mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, theta) -> None:
        th = np.ascontiguousarray(theta, dtype=np.float32)
        assert th.size == self.nparam
        _check(self.lib, self.lib.nce_mlp_set_params(self.h, th.ctypes.data))

    def _run(self, fn):
        torch = self.torch
        self.stream.wait_stream(torch.cuda.current_stream())
        r = fn(ctypes.c_void_p(self.stream.cuda_stream))
        torch.cuda.current_stream().wait_stream(self.stream)
        return r

    def forward(self, x):
        torch = self.torch
        y = torch.empty((x.shape[0], self.shape[3]), dtype=torch.float32, device="cuda")
        self._run(lambda st: _check(self.lib, self.lib.nce_mlp_forward(
            self.h, _ptr(x, torch.float32), x.shape[0], _ptr(y, torch.float32), st)))
        return y

    def forward_noalloc(self, x, y):
        """nce_mlp_forward_noalloc into the caller's y (B x n_out FP32 CUDA
        tensor): no device allocation inside the library."""
        torch = self.torch
        self._run(lambda st: _check(self.lib, self.lib.nce_mlp_forward_noalloc(
            self.h, _ptr(x, torch.float32), x.shape[0], _ptr(y, torch.float32), st)))
        return y

    def loss_grad(self, x, t):
        torch = self.torch
        loss = ctypes.c_double()
        g = np.empty(self.nparam, dtype=np.float32)
        self._run(lambda st: _check(self.lib, self.lib.nce_mlp_loss_grad(
            self.h, _ptr(x, torch.float32), _ptr(t, torch.float32), x.shape[0], ctypes.byref(loss),
            g.ctypes.data, st)))
        return loss.value, g

    def train_step(self, x, t, lr: float) -> float:
        torch = self.torch
        loss = ctypes.c_double()
        self._run(lambda st: _check(self.lib, self.lib.nce_mlp_train_step(
            self.h, _ptr(x, torch.float32), _ptr(t, torch.float32), x.shape[0], float(lr), ctypes.byref(loss), st)))
        return loss.value


class Context:
    """One patch layout on the current HIP device (nce_setup ... nce_destroy).
    eps: the common patch radius, or one radius per patch (several radii:
    nce_setup_radii)."""

    def __init__(self, centers: np.ndarray, eps: float, problem: int = INTERIOR, M: int = 15,
                 tol_id: float = 1e-11, tol_grid: float = 1e-8, tol_gmres: float = 1e-10,
                 max_iter: int = 100, precision: int = FP64, far_field: int = FAR_AUTO,
                 cache_dir: Optional[str] = None, stream=None, tol_grid_fp32: Optional[float] = None,
                 tol_id_fp32: Optional[float] = None, tol_coarse: Optional[float] = None,
                 deflation: Optional[bool] = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs only on the GPU")
        self.lib = load()
        self.torch = torch
        c = np.ascontiguousarray(centers, dtype=np.float64)
        o = Opts()
        self.lib.nce_default_opts(ctypes.byref(o))
        o.problem, o.M, o.tol_id, o.tol_grid, o.tol_gmres = problem, M, tol_id, tol_grid, tol_gmres
        if tol_grid_fp32 is not None:
            o.tol_grid_fp32 = tol_grid_fp32
        if tol_id_fp32 is not None:
            o.tol_id_fp32 = tol_id_fp32
        if tol_coarse is not None:
            o.tol_coarse = tol_coarse
        if deflation is not None:
            o.deflation = int(bool(deflation))
        o.max_iter, o.precision, o.far_field = max_iter, precision, far_field
        # the library works on its own (non-default) stream; calls below order
        # it against the caller's current stream in both directions
        self.stream = stream if stream is not None else torch.cuda.Stream()
        o.stream = ctypes.c_void_p(self.stream.cuda_stream)
        self._cache = (cache_dir or os.environ.get("NCE_CACHE") or "").encode() or None
        o.cache_dir = self._cache
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        if np.ndim(eps) == 0:
            _check(self.lib, self.lib.nce_setup(c.ctypes.data, len(c), float(eps), ctypes.byref(o), ctypes.byref(h)))
            self.eps = float(eps)
        else:
            r = np.ascontiguousarray(eps, dtype=np.float64)
            if r.shape != (len(c),):
                raise ValueError("one radius per patch expected")
            _check(self.lib, self.lib.nce_setup_radii(c.ctypes.data, r.ctypes.data, len(c), ctypes.byref(o),
                                                      ctypes.byref(h)))
            self.eps = r.copy()
        self.h = h
        self.N = len(c)
        self.problem = problem
        K, Ks, p, L = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib, self.lib.nce_dims(h, ctypes.byref(K), ctypes.byref(Ks), ctypes.byref(p), ctypes.byref(L)))
        self.K, self.Kstar, self.p, self.levels = K.value, Ks.value, p.value, L.value

    def close(self):
        if getattr(self, "h", None):
            self.lib.nce_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def frames(self) -> np.ndarray:
        out = np.empty((self.N, 9))
        _check(self.lib, self.lib.nce_frames(self.h, out.ctypes.data))
        return out

    def integral_vector(self) -> np.ndarray:
        out = np.empty(self.K)
        _check(self.lib, self.lib.nce_integral_vector(self.h, out.ctypes.data))
        return out

    def types(self):
        """nce_types: (radii, integral vectors (one row per radius), type of every patch)."""
        n = ctypes.c_int()
        eps = np.empty(8)
        I = np.empty((8, self.K))
        t = np.empty(self.N, dtype=np.int32)
        _check(self.lib, self.lib.nce_types(self.h, ctypes.byref(n), eps.ctypes.data, I.ctypes.data, t.ctypes.data))
        return eps[:n.value].copy(), I[:n.value].copy(), t

    def field(self, coeffs, points, physical: bool = False):
        """nce_field: the potential u / v (or, physical=True, ubar / vbar) at
        points (n x 3 float64 CUDA tensor) for coefficients (N K float64 CUDA
        tensor)."""
        torch = self.torch
        pts = points.reshape(-1, 3)
        out = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
        self._enter()
        _check(self.lib, self.lib.nce_field(self.h, _ptr(coeffs), _ptr(pts), pts.shape[0], int(bool(physical)),
                                            _ptr(out)))
        self._leave()
        return out

    def patch_residual(self, coeffs, patches, n_t: int = 20, n_theta: int = 40) -> np.ndarray:
        """nce_patch_residual: (1/|Gamma_i|) ||v - 1||_L2 on each listed patch."""
        idx = np.ascontiguousarray(np.atleast_1d(patches), dtype=np.int64)
        out = np.empty(len(idx))
        self._enter()
        _check(self.lib, self.lib.nce_patch_residual(self.h, _ptr(coeffs), idx.ctypes.data, len(idx), int(n_t),
                                                     int(n_theta), out.ctypes.data))
        self._leave()
        return out

    def work(self, precision: int = FP64):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self.lib, self.lib.nce_work(self.h, int(precision), ctypes.byref(a), ctypes.byref(b),
                                           ctypes.byref(c)))
        return {"pairs_far": a.value, "pairs_near": b.value, "interp_fma": c.value}

    def empty(self):
        return self.torch.empty((self.N, self.K), dtype=self.torch.float64, device="cuda")

    def _enter(self):
        self.stream.wait_stream(self.torch.cuda.current_stream())

    def _leave(self):
        self.torch.cuda.current_stream().wait_stream(self.stream)

    def matvec(self, x, y=None, precision: int = FP64):
        """y = A x (device tensors N x K, float64); asynchronous, ordered after
        the caller's current stream and before its later work."""
        if y is None:
            y = self.empty()
        self._enter()
        _check(self.lib, self.lib.nce_matvec(self.h, _ptr(x), _ptr(y), int(precision)))
        self._leave()
        return y

    def matvec_profile(self, x, y=None, precision: int = FP64):
        """y = A x with per-step times in ms: [block apply, far, near, interpolation, P apply]."""
        if y is None:
            y = self.empty()
        ms = np.zeros(5)
        self._enter()
        _check(self.lib, self.lib.nce_matvec_profile(self.h, _ptr(x), _ptr(y), int(precision), ms.ctypes.data))
        self._leave()
        return y, ms

    def features(self):
        f = self.torch.empty((self.N, FEATURES), dtype=self.torch.float32, device="cuda")
        self._enter()
        _check(self.lib, self.lib.nce_features(self.h, _ptr(f, self.torch.float32)))
        self._leave()
        return f

    def set_warm_start(self, mlp: Optional["Mlp"] = None, coarse: bool = True) -> None:
        """Start later solves from the coarse solve (coarse=True), refined by the
        network when one is given; set_warm_start(None, False) disables."""
        self._warm = mlp  # keep the network alive while it is set
        _check(self.lib, self.lib.nce_set_warm_start(self.h, mlp.h if mlp is not None else None, int(bool(coarse))))

    def coarse(self, with_chi0: bool = False):
        """(coarse amplitudes a as an N float64 device tensor in the caller's
        patch order, GMRES iterations [, chi0]); chi0 is a float for one patch
        radius and an array of one value per radius (order of types()) for
        several."""
        a = self.torch.empty(self.N, dtype=self.torch.float64, device="cuda")
        it = ctypes.c_int()
        chi0 = np.zeros(8)
        self._enter()
        _check(self.lib, self.lib.nce_coarse_solve(self.h, _ptr(a), ctypes.byref(it), chi0.ctypes.data_as(
            ctypes.POINTER(ctypes.c_double))))
        self._leave()
        if not with_chi0:
            return a, it.value
        nt = len(self.types()[0])
        return a, it.value, (float(chi0[0]) if nt == 1 else chi0[:nt].copy())

    def set_deflation(self, on: bool) -> None:
        _check(self.lib, self.lib.nce_set_deflation(self.h, int(bool(on))))

    def deflation_matrix(self):
        """(k, T): the coarse operator of the mixed solves' deflation on its k
        basis columns (k x k numpy array; k = 0 for N < 64)."""
        k = ctypes.c_int()
        T = np.zeros(256)
        self._enter()
        _check(self.lib, self.lib.nce_deflation_matrix(self.h, ctypes.byref(k), T.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        self._leave()
        return k.value, T[:k.value * k.value].reshape(k.value, k.value)

    def set_shapes(self, precision: int, p2l: int, l2t: int) -> None:
        """nce_set_shapes: far-field kernel shapes (P2L 0, 4, 8 or 16; interpolation 2, 4 or 8)."""
        _check(self.lib, self.lib.nce_set_shapes(self.h, int(precision), int(p2l), int(l2t)))

    def set_solver(self, tol_gmres: float, max_iter: int, precision: int):
        _check(self.lib, self.lib.nce_set_solver(self.h, float(tol_gmres), int(max_iter), int(precision)))

    def autotune(self, precision: int = FP64):
        """Pick the fastest far-field kernel shapes on this layout; returns
        (P2L grid points per thread, interpolation nodes per thread)."""
        ch = np.zeros(2, dtype=np.int32)
        _check(self.lib, self.lib.nce_autotune(self.h, int(precision), ch.ctypes.data))
        return int(ch[0]), int(ch[1])

    def solve(self, want_coeffs: bool = True, want_flux: bool = True) -> dict:
        x = self.empty() if want_coeffs else None
        f = self.torch.empty(self.N, dtype=self.torch.float64, device="cuda") if want_flux else None
        info = Info()
        out = {}
        self._enter()
        if self.problem == INTERIOR:
            mu = ctypes.c_double()
            rc = self.lib.nce_solve_interior(self.h, _ptr(x), _ptr(f), ctypes.byref(mu), ctypes.byref(info))
            _check(self.lib, rc, allow_notconv=True)
            out["mu"] = mu.value
        else:
            rate, Is = ctypes.c_double(), ctypes.c_double()
            rc = self.lib.nce_solve_exterior(self.h, _ptr(x), _ptr(f), ctypes.byref(rate), ctypes.byref(Is),
                                             ctypes.byref(info))
            _check(self.lib, rc, allow_notconv=True)
            out["capture_rate"] = rate.value
            out["I_sigma"] = Is.value
        self._leave()
        out.update(info.asdict())
        out["converged"] = rc == 0
        out["x"] = x
        out["flux"] = f
        return out


class Batch:
    """Independent configurations solved together (nce_setup_batch ...
    nce_destroy_batch). configs: sequence of (centers N_b x 3, eps_b, problem_b).
    Batch vectors are flat float64 device tensors of length n; configuration b
    occupies [offsets[b], offsets[b] + N_b K)."""

    def __init__(self, configs, M: int = 15, tol_id: float = 1e-11, tol_grid: float = 1e-8,
                 tol_gmres: float = 1e-10, max_iter: int = 60, precision: int = MIXED, far_field: int = FAR_AUTO,
                 cache_dir: Optional[str] = None, stream=None, tol_grid_fp32: Optional[float] = None,
                 tol_id_fp32: Optional[float] = None, tol_coarse: Optional[float] = None,
                 deflation: Optional[bool] = None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device: the solver runs only on the GPU")
        self.lib = load()
        self.torch = torch
        cs = [np.ascontiguousarray(c, dtype=np.float64) for c, _, _ in configs]
        self.B = len(cs)
        self.N = np.array([len(c) for c in cs], dtype=np.int64)
        self.eps = np.array([float(e) for _, e, _ in configs], dtype=np.float64)
        self.problem = np.array([int(p) for _, _, p in configs], dtype=np.int32)
        ptrs = (ctypes.c_void_p * self.B)(*[c.ctypes.data for c in cs])
        o = Opts()
        self.lib.nce_default_opts(ctypes.byref(o))
        o.M, o.tol_id, o.tol_grid, o.tol_gmres = M, tol_id, tol_grid, tol_gmres
        if tol_grid_fp32 is not None:
            o.tol_grid_fp32 = tol_grid_fp32
        if tol_id_fp32 is not None:
            o.tol_id_fp32 = tol_id_fp32
        if tol_coarse is not None:
            o.tol_coarse = tol_coarse
        if deflation is not None:
            o.deflation = int(bool(deflation))
        o.max_iter, o.precision, o.far_field = max_iter, precision, far_field
        self.stream = stream if stream is not None else torch.cuda.Stream()
        o.stream = ctypes.c_void_p(self.stream.cuda_stream)
        self._cache = (cache_dir or os.environ.get("NCE_CACHE") or "").encode() or None
        o.cache_dir = self._cache
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(self.lib, self.lib.nce_setup_batch(ptrs, self.N.ctypes.data, self.eps.ctypes.data,
                                                  self.problem.ctypes.data, self.B, ctypes.byref(o),
                                                  ctypes.byref(h)))
        self.h = h
        n, K, G = ctypes.c_int64(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib, self.lib.nce_batch_dims(h, ctypes.byref(n), ctypes.byref(K), ctypes.byref(G)))
        self.n, self.K, self.ngroups = n.value, K.value, G.value
        self.offsets = np.zeros(self.B, dtype=np.int64)
        self.far_tree = np.zeros(self.B, dtype=np.int32)
        _check(self.lib, self.lib.nce_batch_offsets(h, self.offsets.ctypes.data, self.far_tree.ctypes.data))

    def close(self):
        if getattr(self, "h", None):
            self.lib.nce_destroy_batch(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        return self.torch.empty(self.n, dtype=self.torch.float64, device="cuda")

    def part(self, v, b: int):
        """View of configuration b's N_b x K block of a batch vector."""
        o = int(self.offsets[b])
        return v[o:o + int(self.N[b]) * self.K].view(int(self.N[b]), self.K)

    def types(self):
        """nce_types: (radii, integral vectors (one row per radius), type of every patch)."""
        n = ctypes.c_int()
        eps = np.empty(8)
        I = np.empty((8, self.K))
        t = np.empty(self.N, dtype=np.int32)
        _check(self.lib, self.lib.nce_types(self.h, ctypes.byref(n), eps.ctypes.data, I.ctypes.data, t.ctypes.data))
        return eps[:n.value].copy(), I[:n.value].copy(), t

    def field(self, coeffs, points, physical: bool = False):
        """nce_field: the potential u / v (or, physical=True, ubar / vbar) at
        points (n x 3 float64 CUDA tensor) for coefficients (N K float64 CUDA
        tensor)."""
        torch = self.torch
        pts = points.reshape(-1, 3)
        out = torch.empty(pts.shape[0], dtype=torch.float64, device="cuda")
        self._enter()
        _check(self.lib, self.lib.nce_field(self.h, _ptr(coeffs), _ptr(pts), pts.shape[0], int(bool(physical)),
                                            _ptr(out)))
        self._leave()
        return out

    def patch_residual(self, coeffs, patches, n_t: int = 20, n_theta: int = 40) -> np.ndarray:
        """nce_patch_residual: (1/|Gamma_i|) ||v - 1||_L2 on each listed patch."""
        idx = np.ascontiguousarray(np.atleast_1d(patches), dtype=np.int64)
        out = np.empty(len(idx))
        self._enter()
        _check(self.lib, self.lib.nce_patch_residual(self.h, _ptr(coeffs), idx.ctypes.data, len(idx), int(n_t),
                                                     int(n_theta), out.ctypes.data))
        self._leave()
        return out

    def work(self, precision: int = FP64):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self.lib, self.lib.nce_batch_work(self.h, int(precision), ctypes.byref(a), ctypes.byref(b),
                                                 ctypes.byref(c)))
        return {"pairs_far": a.value, "pairs_near": b.value, "interp_fma": c.value}

    def matvec(self, x, y=None, precision: int = FP64):
        if y is None:
            y = self.empty()
        self.stream.wait_stream(self.torch.cuda.current_stream())
        _check(self.lib, self.lib.nce_batch_matvec(self.h, _ptr(x), _ptr(y), int(precision)))
        self.torch.cuda.current_stream().wait_stream(self.stream)
        return y

    def set_solver(self, tol_gmres: float, max_iter: int, precision: int, use_graph: bool = True):
        _check(self.lib, self.lib.nce_batch_set_solver(self.h, float(tol_gmres), int(max_iter), int(precision),
                                                       int(bool(use_graph))))

    def set_warm_start(self, mlp: Optional["Mlp"] = None, coarse: bool = True) -> None:
        """Start later batched solves from per-member coarse solves (refined by
        the network when given); set_warm_start(None, False) disables."""
        self._warm = mlp
        _check(self.lib, self.lib.nce_batch_set_warm_start(self.h, mlp.h if mlp is not None else None,
                                                           int(bool(coarse))))

    def set_deflation(self, on: bool) -> None:
        """nce_batch_set_deflation: deflation of the mixed inner solves per member."""
        _check(self.lib, self.lib.nce_batch_set_deflation(self.h, int(bool(on))))

    def autotune(self, precision: int = MIXED):
        """nce_batch_autotune: per group (P2L points per thread, interpolation nodes per thread)."""
        ch = np.zeros(2 * self.ngroups, dtype=np.int32)
        _check(self.lib, self.lib.nce_batch_autotune(self.h, int(precision), ch.ctypes.data))
        return [(int(ch[2 * g]), int(ch[2 * g + 1])) for g in range(self.ngroups)]

    def solve(self, want_coeffs: bool = False) -> dict:
        x = self.empty() if want_coeffs else None
        res = np.zeros(self.B)
        infos = (Info * self.B)()
        self.stream.wait_stream(self.torch.cuda.current_stream())
        rc = self.lib.nce_solve_batch(self.h, res.ctypes.data, _ptr(x), infos)
        _check(self.lib, rc, allow_notconv=True)
        self.torch.cuda.current_stream().wait_stream(self.stream)
        return {"result": res, "info": [infos[b].asdict() for b in range(self.B)], "converged": rc == 0, "x": x}
