"""ctypes binding of libgmg.so (the C ABI in include/gmg.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Tensors are torch CUDA (HIP) tensors, float64, contiguous; the
library works on torch's current stream.  If the library is not built the
first call raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gmg.h")

STATUS = {0: "GMG_OK", 1: "GMG_ERR_ARG", 2: "GMG_ERR_DIMS", 3: "GMG_ERR_COEFF", 4: "GMG_ERR_NOMEM",
          5: "GMG_ERR_HIP", 6: "GMG_ERR_NOT_CONVERGED", 7: "GMG_ERR_BREAKDOWN"}
OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN = 0, 6, 7
FP64, MIXED = 0, 1
COARSE_ARITHMETIC, COARSE_HARMONIC = 0, 1


class Options(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("levels", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double), ("switch_n", ctypes.c_int32),
                ("persistent_wgs", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("coarse_rule", ctypes.c_int32), ("coeff_is_log", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("coarse_solver", ctypes.c_int32),
                ("coarse_rtol", ctypes.c_double), ("coarse_max_it", ctypes.c_int32),
                ("flexible", ctypes.c_int32), ("switch2_n", ctypes.c_int32),
                ("galerkin", ctypes.c_int32), ("persistent_lds", ctypes.c_int32),
                ("post_fused", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("restarts", ctypes.c_int32), ("rel_res", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("setup_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("coarse_iterations", ctypes.c_int32)]

    def as_dict(self, status: int):
        return {"status": STATUS.get(status, str(status)), "iterations": self.iterations,
                "restarts": self.restarts, "rel_res": self.rel_res, "rel_res_true": self.rel_res_true,
                "setup_ms": self.setup_ms, "solve_ms": self.solve_ms, "coarse_iterations": self.coarse_iterations}


class GmgError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def declared_functions():
    """Names of the functions include/gmg.h declares."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gmg_[a-z_0-9]+)\s*\(", src)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1604_07163_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    st = ctypes.c_int
    L.gmg_default_options.argtypes = [ctypes.POINTER(Options), I32]
    L.gmg_default_options.restype = None
    L.gmg_create.argtypes = [ctypes.POINTER(Options), P, P, P, P, ctypes.POINTER(P)]
    L.gmg_create.restype = st
    L.gmg_set_coefficients.argtypes = [P, P, P, P]
    L.gmg_set_coefficients.restype = st
    L.gmg_set_stream.argtypes = [P, P]
    L.gmg_set_stream.restype = st
    L.gmg_solve.argtypes = [P, P, P, P, D, I32, ctypes.POINTER(Info)]
    L.gmg_solve.restype = st
    L.gmg_adjoint_gradient.argtypes = [P, P, P, P, P, P, P, D, I32, ctypes.POINTER(Info)]
    L.gmg_adjoint_gradient.restype = st
    L.gmg_level_n.argtypes = [P, I32]
    L.gmg_level_n.restype = I32
    L.gmg_apply_operator.argtypes = [P, I32, P, P]
    L.gmg_apply_operator.restype = st
    L.gmg_apply_outer_operator.argtypes = [P, P, P]
    L.gmg_apply_outer_operator.restype = st
    L.gmg_debug_smooth.argtypes = [P, I32, P, P, I32]
    L.gmg_debug_smooth.restype = st
    L.gmg_debug_residual_restrict.argtypes = [P, I32, P, P, P]
    L.gmg_debug_residual_restrict.restype = st
    L.gmg_debug_prolong.argtypes = [P, I32, P, P]
    L.gmg_debug_prolong.restype = st
    L.gmg_debug_coarse_solve.argtypes = [P, P, P]
    L.gmg_debug_coarse_solve.restype = st
    L.gmg_debug_vcycle.argtypes = [P, P, P]
    L.gmg_debug_vcycle.restype = st
    L.gmg_get_level_coefficients.argtypes = [P, I32, P, P, P]
    L.gmg_get_level_coefficients.restype = st
    L.gmg_get_level_stencil.argtypes = [P, I32, P]
    L.gmg_get_level_stencil.restype = st
    L.gmg_get_level_interval.argtypes = [P, I32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.gmg_persistent_lds_bytes.argtypes = [P]
    L.gmg_persistent_lds_bytes.restype = ctypes.c_uint64
    L.gmg_get_level_interval.restype = st
    L.gmg_profile_start.argtypes = [P]
    L.gmg_profile_start.restype = st
    L.gmg_profile_stop.argtypes = [P]
    L.gmg_profile_stop.restype = st
    L.gmg_profile_get.argtypes = [P, I32, ctypes.POINTER(I32), ctypes.POINTER(D)]
    L.gmg_profile_get.restype = st
    L.gmg_kernel_class_name.argtypes = [I32]
    L.gmg_kernel_class_name.restype = ctypes.c_char_p
    L.gmg_calibration_copy.argtypes = [P, P, ctypes.c_uint64, ctypes.c_int32, P]
    L.gmg_calibration_copy.restype = st
    L.gmg_solve_static.argtypes = [ctypes.POINTER(Options), P, P, P, P, P, P, D, I32, P, ctypes.POINTER(Info)]
    L.gmg_solve_static.restype = st
    L.gmg_destroy.argtypes = [P]
    L.gmg_destroy.restype = None
    L.gmg_status_string.argtypes = [st]
    L.gmg_status_string.restype = ctypes.c_char_p
    L.gmg_last_error.argtypes = [P]
    L.gmg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _dev(t: torch.Tensor, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    return ctypes.c_void_p(t.data_ptr())


def face_shapes(n: int):
    return (n, n, n - 1), (n, n - 1, n), (n - 1, n, n)


def default_levels(n: int) -> int:
    lv, t = 0, n - 1
    while t > 1 and t % 2 == 0:
        lv += 1
        t //= 2
    return max(lv, 1)


class Solver:
    """A hierarchy on the GPU plus its solver state (one handle).

    kx, ky, kz: CUDA float64 link coefficients (shapes (N,N,N-1), (N,N-1,N),
    (N-1,N,N); ln k with coeff_is_log).  Keyword options map one to one onto
    gmg_options in include/gmg.h: levels (default log2(N-1)), precision
    ("fp64" | "mixed"), switch_n (persistent coarse kernel for N_l <= switch_n,
    0 = off), persistent_wgs / switch2_n (a team of workgroups, two-stage),
    persistent_lds, coarse_rule ("arithmetic" | "harmonic"), cheb_degree /
    cheb_lo / cheb_hi, coarse_solver ("exact" | "cg") with coarse_rtol /
    coarse_max_it, flexible (Polak-Ribiere beta), galerkin (first Galerkin
    level, 0 = none), post_fused ("auto" | True | False), check_every.
    """

    def __init__(self, kx, ky, kz, *, levels=None, precision="fp64", switch_n=0, coarse_rule="arithmetic",
                 cheb_degree=2, cheb_lo=0.25, cheb_hi=2.0, coeff_is_log=False, check_every=0,
                 persistent_wgs=1, coarse_solver="exact", coarse_rtol=1e-4, coarse_max_it=500, flexible=False,
                 switch2_n=0, galerkin=0, persistent_lds=True, post_fused="auto"):
        L = lib()
        n = int(kx.shape[0])
        self.n = n
        o = Options()
        L.gmg_default_options(ctypes.byref(o), n)
        o.levels = default_levels(n) if levels is None else int(levels)
        o.cheb_degree = cheb_degree
        o.cheb_lo = cheb_lo
        o.cheb_hi = cheb_hi
        o.switch_n = int(switch_n)
        o.persistent_wgs = int(persistent_wgs)
        o.precision = {"fp64": FP64, "mixed": MIXED}[precision] if isinstance(precision, str) else int(precision)
        o.coarse_rule = ({"arithmetic": COARSE_ARITHMETIC, "harmonic": COARSE_HARMONIC}[coarse_rule]
                         if isinstance(coarse_rule, str) else int(coarse_rule))
        o.coeff_is_log = 1 if coeff_is_log else 0
        o.check_every = int(check_every)
        o.coarse_solver = ({"exact": 0, "cg": 1}[coarse_solver] if isinstance(coarse_solver, str)
                           else int(coarse_solver))
        o.coarse_rtol = float(coarse_rtol)
        o.coarse_max_it = int(coarse_max_it)
        o.flexible = 1 if flexible else 0
        o.switch2_n = int(switch2_n)
        o.galerkin = int(galerkin)
        o.persistent_lds = 1 if persistent_lds else 0
        o.post_fused = 2 if post_fused == "auto" else (1 if post_fused else 0)
        self.options = o
        self.levels = o.levels
        self._h = ctypes.c_void_p()
        self._check_faces(kx, ky, kz)
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        s = L.gmg_create(ctypes.byref(o), _dev(kx, "kx"), _dev(ky, "ky"), _dev(kz, "kz"), stream,
                         ctypes.byref(self._h))
        if s != OK:
            raise GmgError(s, "gmg_create")
        self.version = 0

    # ------------------------------------------------------------------ helpers
    def _check_faces(self, kx, ky, kz):
        for t, shp, nm in zip((kx, ky, kz), face_shapes(self.n), ("kx", "ky", "kz")):
            if tuple(t.shape) != shp:
                raise ValueError(f"{nm} must have shape {shp}, got {tuple(t.shape)}")

    def _vec(self, t, name, level=0):
        n = self.level_n(level)
        if tuple(t.shape) != (n, n, n):
            raise ValueError(f"{name} must have shape {(n, n, n)}")
        return _dev(t, name)

    def _err(self, s, what):
        msg = lib().gmg_last_error(self._h)
        raise GmgError(s, f"{what}: {msg.decode() if msg else ''}")

    def _sync_stream(self):
        lib().gmg_set_stream(self._h, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))

    def _empty(self, n):
        return torch.empty((n, n, n), dtype=torch.float64, device="cuda")

    # ------------------------------------------------------------------ API
    def close(self):
        if self._h:
            lib().gmg_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_n(self, level: int) -> int:
        return lib().gmg_level_n(self._h, level)

    def set_coefficients(self, kx, ky, kz):
        """Rebuild the hierarchy from new coefficients (enqueued on the stream;
        a bad k is reported by the next solve as GMG_ERR_COEFF)."""
        self._check_faces(kx, ky, kz)
        self._sync_stream()
        s = lib().gmg_set_coefficients(self._h, _dev(kx, "kx"), _dev(ky, "ky"), _dev(kz, "kz"))
        if s != OK:
            self._err(s, "gmg_set_coefficients")
        self.version += 1

    def solve(self, f, rtol=1e-8, max_it=500, x0=None, out=None, raise_on_failure=False):
        """Returns (x, info).  info["status"] is GMG_OK, GMG_ERR_NOT_CONVERGED or GMG_ERR_BREAKDOWN."""
        self._sync_stream()
        x = self._empty(self.n) if out is None else out
        info = Info()
        s = lib().gmg_solve(self._h, self._vec(f, "f"), self._vec(x, "x"),
                            None if x0 is None else self._vec(x0, "x0"), float(rtol), int(max_it),
                            ctypes.byref(info))
        if s not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN) or (raise_on_failure and s != OK):
            self._err(s, "gmg_solve")
        return x, info.as_dict(s)

    def adjoint_gradient(self, phi, dl_dphi, rtol=1e-10, max_it=500, want_lambda=True):
        """Returns (g_x, g_y, g_z, lambda, info): g = dL/d(ln k) on the three link arrays."""
        self._sync_stream()
        sx, sy, sz = face_shapes(self.n)
        gx = torch.empty(sx, dtype=torch.float64, device="cuda")
        gy = torch.empty(sy, dtype=torch.float64, device="cuda")
        gz = torch.empty(sz, dtype=torch.float64, device="cuda")
        lam = self._empty(self.n) if want_lambda else None
        info = Info()
        s = lib().gmg_adjoint_gradient(self._h, self._vec(phi, "phi"), self._vec(dl_dphi, "dl_dphi"),
                                       _dev(gx, "g_x"), _dev(gy, "g_y"), _dev(gz, "g_z"),
                                       None if lam is None else self._vec(lam, "lambda"), float(rtol),
                                       int(max_it), ctypes.byref(info))
        if s not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN):
            self._err(s, "gmg_adjoint_gradient")
        return gx, gy, gz, lam, info.as_dict(s)

    # ------------------------------------------------------------------ test hooks
    def apply_operator(self, level, x, use_fp64=False):
        """y = A_l x in the V-cycle precision; use_fp64 (level 0 only): the
        outer FP64 operator of the CG iteration."""
        self._sync_stream()
        y = self._empty(self.level_n(level))
        if use_fp64:
            if level != 0:
                raise ValueError("the outer FP64 operator exists on level 0 only")
            s = lib().gmg_apply_outer_operator(self._h, self._vec(x, "x"), _dev(y, "y"))
            if s != OK:
                self._err(s, "gmg_apply_outer_operator")
            return y
        s = lib().gmg_apply_operator(self._h, level, self._vec(x, "x", level), _dev(y, "y"))
        if s != OK:
            self._err(s, "gmg_apply_operator")
        return y

    def smooth(self, level, b, x0=None):
        self._sync_stream()
        n = self.level_n(level)
        x = torch.zeros((n, n, n), dtype=torch.float64, device="cuda") if x0 is None else x0.clone()
        s = lib().gmg_debug_smooth(self._h, level, self._vec(b, "b", level), _dev(x, "x"),
                                   1 if x0 is None else 0)
        if s != OK:
            self._err(s, "gmg_debug_smooth")
        return x

    def residual_restrict(self, level, b, x):
        self._sync_stream()
        bc = self._empty(self.level_n(level + 1))
        s = lib().gmg_debug_residual_restrict(self._h, level, self._vec(b, "b", level), self._vec(x, "x", level),
                                              _dev(bc, "b_coarse"))
        if s != OK:
            self._err(s, "gmg_debug_residual_restrict")
        return bc

    def prolong(self, level, e, x):
        self._sync_stream()
        out = x.clone()
        s = lib().gmg_debug_prolong(self._h, level, self._vec(e, "e", level + 1), self._vec(out, "x", level))
        if s != OK:
            self._err(s, "gmg_debug_prolong")
        return out

    def coarse_solve(self, b):
        self._sync_stream()
        lc = self.levels - 1
        x = self._empty(self.level_n(lc))
        s = lib().gmg_debug_coarse_solve(self._h, self._vec(b, "b", lc), _dev(x, "x"))
        if s != OK:
            self._err(s, "gmg_debug_coarse_solve")
        return x

    def vcycle(self, r):
        self._sync_stream()
        z = self._empty(self.n)
        s = lib().gmg_debug_vcycle(self._h, self._vec(r, "r"), _dev(z, "z"))
        if s != OK:
            self._err(s, "gmg_debug_vcycle")
        return z

    def level_coefficients(self, level):
        self._sync_stream()
        n = self.level_n(level)
        sx, sy, sz = face_shapes(n)
        kx = torch.empty(sx, dtype=torch.float64, device="cuda")
        ky = torch.empty(sy, dtype=torch.float64, device="cuda")
        kz = torch.empty(sz, dtype=torch.float64, device="cuda")
        s = lib().gmg_get_level_coefficients(self._h, level, _dev(kx, "kx"), _dev(ky, "ky"), _dev(kz, "kz"))
        if s != OK:
            self._err(s, "gmg_get_level_coefficients")
        return kx, ky, kz

    @property
    def persistent_lds_bytes(self):
        """LDS bytes of the one-workgroup persistent kernel, 0 when it runs from HBM/L2."""
        return int(lib().gmg_persistent_lds_bytes(self._h))

    def level_interval(self, level):
        """Chebyshev interval (lo, hi) of D^-1 A the smoother uses on `level`."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        s = lib().gmg_get_level_interval(self._h, level, ctypes.byref(lo), ctypes.byref(hi))
        if s != OK:
            self._err(s, "gmg_get_level_interval")
        return lo.value, hi.value

    def level_stencil(self, level):
        """FP64 Galerkin operator of `level` as an (N, N, N, 27) tensor, entry
        (dz+1)*9 + (dy+1)*3 + (dx+1) the coefficient of u(i+dx, j+dy, k+dz)."""
        self._sync_stream()
        n = self.level_n(level)
        out = torch.empty((n, n, n, 27), dtype=torch.float64, device="cuda")
        s = lib().gmg_get_level_stencil(self._h, level, _dev(out, "a27"))
        if s != OK:
            self._err(s, "gmg_get_level_stencil")
        return out


KERNEL_CLASSES = ["apply_dot", "residual", "update_r", "update_p", "cheb_first", "cheb_step", "cheb_step_prev",
                  "cheb_step_dot", "level_residual", "prolong", "persistent", "coarse_solve", "face_gradient",
                  "restrict", "update_xp", "cheb_pre2", "cheb_post2", "pre2_res"]


class Profile:
    """Context manager: per-kernel-class launch counts and device time (HIP events)."""

    def __init__(self, solver: "Solver"):
        self.solver = solver
        self.result = {}

    def __enter__(self):
        self.solver._sync_stream()
        s = lib().gmg_profile_start(self.solver._h)
        if s != OK:
            self.solver._err(s, "gmg_profile_start")
        return self

    def __exit__(self, *exc):
        L = lib()
        L.gmg_profile_stop(self.solver._h)
        for c, name in enumerate(KERNEL_CLASSES):
            n = ctypes.c_int32(0)
            ms = ctypes.c_double(0.0)
            s = L.gmg_profile_get(self.solver._h, c, ctypes.byref(n), ctypes.byref(ms))
            if s != OK:
                self.solver._err(s, "gmg_profile_get")
            if n.value:
                self.result[name] = {"launches": n.value, "total_ms": ms.value, "avg_ms": ms.value / n.value}
        return False


def solve_static(kx, ky, kz, f, *, levels=None, precision="fp64", switch_n=0, persistent_wgs=1, rtol=1e-8,
                 max_it=500, x0=None, out=None, cheb_degree=2, coarse_rule="arithmetic"):
    """gmg_solve_static: build the hierarchy in the library's static device
    workspace and solve, allocating nothing in the library (N <= 65).
    Returns (x, info); raises GmgError for statuses other than the solve's."""
    n = int(kx.shape[0])
    for t, shp, nm in zip((kx, ky, kz), face_shapes(n), ("kx", "ky", "kz")):
        if tuple(t.shape) != shp:
            raise ValueError(f"{nm} must have shape {shp}, got {tuple(t.shape)}")
    for t, nm in ((f, "f"), (out, "x"), (x0, "x0")):
        if t is not None and tuple(t.shape) != (n, n, n):
            raise ValueError(f"{nm} must have shape {(n, n, n)}")
    L = lib()
    o = Options()
    L.gmg_default_options(ctypes.byref(o), n)
    o.levels = default_levels(n) if levels is None else int(levels)
    o.precision = {"fp64": FP64, "mixed": MIXED}[precision]
    o.switch_n = int(switch_n)
    o.persistent_wgs = int(persistent_wgs)
    o.cheb_degree = int(cheb_degree)
    o.coarse_rule = {"arithmetic": COARSE_ARITHMETIC, "harmonic": COARSE_HARMONIC}[coarse_rule]
    x = torch.empty((n, n, n), dtype=torch.float64, device="cuda") if out is None else out
    info = Info()
    s = L.gmg_solve_static(ctypes.byref(o), _dev(kx, "kx"), _dev(ky, "ky"), _dev(kz, "kz"), _dev(f, "f"),
                           _dev(x, "x"), None if x0 is None else _dev(x0, "x0"), float(rtol), int(max_it),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(info))
    if s not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN):
        msg = L.gmg_last_error(None)
        raise GmgError(s, f"gmg_solve_static: {msg.decode() if msg else ''}")
    return x, info.as_dict(s)


def calibration_copy(dst: torch.Tensor, src: torch.Tensor, planes: int = 1):
    """dst <- src with the library's streaming copy kernel (same byte count);
    planes > 1 copies in the z-march pattern of the stencil kernels."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (dst.is_cuda and src.is_cuda):
        raise ValueError("calibration_copy: device tensors of equal byte size required")
    s = lib().gmg_calibration_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                   int(planes), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if s != OK:
        raise GmgError(s, "gmg_calibration_copy")


def raw_create(options: Options, kx, ky, kz):
    """gmg_create with an explicit options struct; returns (status, handle)."""
    h = ctypes.c_void_p()
    s = lib().gmg_create(ctypes.byref(options), _dev(kx, "kx"), _dev(ky, "ky"), _dev(kz, "kz"),
                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    return s, h
