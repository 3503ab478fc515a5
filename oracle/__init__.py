"""FP64 CPU oracle for the multigrid-preconditioned CG solve of -div(k grad phi) = f.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The GPU library never imports,
links or calls anything in this package, and this package imports nothing from
the GPU library.

The arithmetic lives in ``gmg_oracle.c`` (plain C loops, FP64); this module only
builds it with gcc and marshals numpy arrays through ctypes.  Hierarchy(...,
precision="mixed") gives the reduced-precision preconditioner of the mixed
mode (rounded coefficients, FP32 V-cycle input/output and search direction),
evaluated in FP64.

Array conventions (C order, x fastest), N vertices per side, h = 1/(N-1):
  vertex vectors  (N, N, N)
  kx              (N, N, N-1)   link (i,j,k)-(i+1,j,k)
  ky              (N, N-1, N)   link (i,j,k)-(i,j+1,k)
  kz              (N-1, N, N)   link (i,j,k)-(i,j,k+1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmg_oracle.c")
_LIB = os.path.join(_HERE, "libgmg_oracle.so")

STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_DIMS", 3: "ERR_COEFF", 4: "ERR_NOMEM",
          6: "ERR_NOT_CONVERGED", 7: "ERR_BREAKDOWN"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (generic x86-64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        D = ctypes.c_double
        L.or_apply_raw.argtypes = [I, P, P, P, P, P]
        L.or_diag_raw.argtypes = [I, P, P, P, P]
        L.or_coarsen_k_raw.argtypes = [I, P, P, P, I, P, P, P, I]
        L.or_restrict_raw.argtypes = [I, P, I, P]
        L.or_prolong_add_raw.argtypes = [I, P, I, P]
        L.or_cheb_raw.argtypes = [I, P, P, P, I, D, D, P, P, I, P]
        L.or_assemble_dense_raw.argtypes = [I, P, P, P, P]
        L.or_cholesky_raw.argtypes = [I, P]
        L.or_cholesky_raw.restype = I
        L.or_chol_solve_raw.argtypes = [I, P, P]
        L.or_create.argtypes = [I, I, I, D, D, I, P, P, P, ctypes.POINTER(P)]
        L.or_create.restype = I
        L.or_create2.argtypes = [I, I, I, D, D, I, I, D, I, P, P, P, ctypes.POINTER(P)]
        L.or_create2.restype = I
        L.or_create3.argtypes = [I, I, I, D, D, I, I, D, I, I, P, P, P, ctypes.POINTER(P)]
        L.or_create3.restype = I
        L.or_apply27_raw.argtypes = [I, P, P, P]
        L.or_galerkin_raw.argtypes = [I, P, P, P, P, I, P]
        L.or_lanczos_max_raw.argtypes = [I, P, P, P, P, I, P]
        L.or_lanczos_max_raw.restype = D
        L.or_level_interval.argtypes = [P, I, ctypes.POINTER(D), ctypes.POINTER(D)]
        L.or_level_interval.restype = I
        L.or_get_a27.argtypes = [P, I, P]
        L.or_get_a27.restype = I
        L.or_pcg2.argtypes = [P, P, P, D, I, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D),
                              ctypes.POINTER(ctypes.c_long)]
        L.or_pcg2.restype = I
        L.or_destroy.argtypes = [P]
        L.or_level_n.argtypes = [P, I]
        L.or_level_n.restype = I
        L.or_get_k.argtypes = [P, I, P, P, P]
        L.or_coarse_solve.argtypes = [P, P, P]
        L.or_vcycle.argtypes = [P, P, P]
        L.or_smooth.argtypes = [P, I, P, P, I]
        L.or_apply.argtypes = [P, I, P, P]
        L.or_pcg.argtypes = [P, P, P, D, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D)]
        L.or_pcg.restype = I
        L.or_adjoint_gradient.argtypes = [P, P, P, P, P, P, P, D, I, ctypes.POINTER(I)]
        L.or_adjoint_gradient.restype = I
        L.or_set_mixed.argtypes = [P]
        L.or_set_mixed.restype = I
        L.or_last_restarts.argtypes = [P]
        L.or_last_restarts.restype = I
        L.or_last_direction.argtypes = [P, P]
        L.or_last_direction.restype = I
        L.or_round_bf16_raw.argtypes = [ctypes.c_size_t, P, P]
        L.or_round_f32.argtypes = [D]
        L.or_round_f32.restype = D
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def face_shapes(n: int):
    return (n, n, n - 1), (n, n - 1, n), (n - 1, n, n)


# --------------------------------------------------------------------------
# level-free routines
# --------------------------------------------------------------------------
def apply(kx, ky, kz, u):
    """(A u) on one grid: 7-point, variable face coefficients, h^-2 scaling."""
    u = _f64(u)
    n = u.shape[0]
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    out = np.empty_like(u)
    lib().or_apply_raw(n, _p(kx), _p(ky), _p(kz), _p(u), _p(out))
    return out


def diag(kx, ky, kz):
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    n = kx.shape[0]
    d = np.empty((n, n, n))
    lib().or_diag_raw(n, _p(kx), _p(ky), _p(kz), _p(d))
    return d


RULE_ARITHMETIC = 0
RULE_HARMONIC = 1


def coarsen_k(kx, ky, kz, rule=RULE_ARITHMETIC):
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    n = kx.shape[0]
    nc = (n - 1) // 2 + 1
    sx, sy, sz = face_shapes(nc)
    cx, cy, cz = np.empty(sx), np.empty(sy), np.empty(sz)
    lib().or_coarsen_k_raw(n, _p(kx), _p(ky), _p(kz), nc, _p(cx), _p(cy), _p(cz), rule)
    return cx, cy, cz


def restrict(r):
    r = _f64(r)
    n = r.shape[0]
    nc = (n - 1) // 2 + 1
    rc = np.empty((nc, nc, nc))
    lib().or_restrict_raw(n, _p(r), nc, _p(rc))
    return rc


def prolong_add(e, x):
    """Return x + P e (x is not modified)."""
    e = _f64(e)
    x = _f64(x).copy()
    lib().or_prolong_add_raw(e.shape[0], _p(e), x.shape[0], _p(x))
    return x


def cheb(kx, ky, kz, b, x0=None, degree=2, lo=0.25, hi=2.0):
    b = _f64(b)
    n = b.shape[0]
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
    work = np.zeros(4 * n ** 3)
    lib().or_cheb_raw(n, _p(kx), _p(ky), _p(kz), degree, lo, hi, _p(b), _p(x),
                      1 if x0 is None else 0, _p(work))
    return x


def round_bf16(a):
    """Round FP64 values to bfloat16 (8 significant bits, ties to even), as FP64."""
    a = _f64(a)
    out = np.empty_like(a)
    lib().or_round_bf16_raw(a.size, _p(a), _p(out))
    return out


def apply27(a27, u):
    """(A u) for a 27-point stencil a27 of shape (N,N,N,27)."""
    u = _f64(u)
    a27 = _f64(a27)
    out = np.empty_like(u)
    lib().or_apply27_raw(u.shape[0], _p(a27), _p(u), _p(out))
    return out


def lanczos_max(kx, ky, kz, a27=None, steps=20):
    """Lanczos estimate of lambda_max(D^-1 A) for the 7-point operator of the links
    (a27 None) or the 27-point operator a27 of shape (N,N,N,27)."""
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    n = kx.shape[0]
    a = None if a27 is None else _f64(a27)
    work = np.empty(4 * n ** 3)
    return lib().or_lanczos_max_raw(n, _p(kx), _p(ky), _p(kz), None if a is None else _p(a), steps, _p(work))


def galerkin(kx, ky, kz, a27=None):
    """R A P (27-point, (Nc,Nc,Nc,27)) of the fine operator given by links or by a27."""
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    n = kx.shape[0]
    nc = (n - 1) // 2 + 1
    out = np.empty((nc, nc, nc, 27))
    a = None if a27 is None else _f64(a27)
    lib().or_galerkin_raw(n, _p(kx), _p(ky), _p(kz), None if a is None else _p(a), nc, _p(out))
    return out


def assemble_dense(kx, ky, kz):
    kx, ky, kz = _f64(kx), _f64(ky), _f64(kz)
    n = kx.shape[0]
    m = (n - 2) ** 3
    A = np.empty((m, m))
    lib().or_assemble_dense_raw(n, _p(kx), _p(ky), _p(kz), _p(A))
    return A


def cholesky(A):
    """Lower Cholesky factor L with A = L L^T (raises if A is not SPD)."""
    A = _f64(A).copy()
    if lib().or_cholesky_raw(A.shape[0], _p(A)) != 0:
        raise np.linalg.LinAlgError("not SPD")
    return np.tril(A)


def chol_solve(L, b):
    L = _f64(L)
    y = _f64(b).copy()
    lib().or_chol_solve_raw(L.shape[0], _p(L), _p(y))
    return y


# --------------------------------------------------------------------------
# hierarchy
# --------------------------------------------------------------------------
class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(STATUS.get(code, str(code)))
        self.code = code


class Hierarchy:
    """Multigrid hierarchy + PCG on the CPU in FP64."""

    def __init__(self, kx, ky, kz, levels: int, degree: int = 2, lo: float = 0.25, hi: float = 2.0,
                 rule: int = RULE_ARITHMETIC, coarse_solver: int = 0, coarse_rtol: float = 1e-4,
                 coarse_max_it: int = 500, galerkin: int = 0, precision: str = "fp64"):
        """coarse_solver 0: exact Cholesky on the coarsest level; 1: truncated
        hierarchy whose coarsest level is solved by Jacobi-CG to coarse_rtol.
        galerkin g > 0: levels l >= g use R A P (True = 1: all coarse levels);
        levels below g keep re-discretized link coefficients.
        precision "mixed": the reduced-precision preconditioner (V-cycle
        coefficients rounded to bfloat16 / FP32, FP32 V-cycle input and output
        and search direction, true-residual restarts), still computed in FP64;
        apply(), smooth() and vcycle() then use the rounded coefficients, the
        outer CG the FP64 ones."""
        if precision not in ("fp64", "mixed"):
            raise ValueError("precision must be 'fp64' or 'mixed'")
        self._kx, self._ky, self._kz = _f64(kx), _f64(ky), _f64(kz)
        self.n = self._kx.shape[0]
        self.levels = levels
        h = ctypes.c_void_p()
        st = lib().or_create3(self.n, levels, degree, lo, hi, rule, coarse_solver, coarse_rtol, coarse_max_it,
                              int(galerkin), _p(self._kx), _p(self._ky), _p(self._kz), ctypes.byref(h))
        if st != 0:
            raise OracleError(st)
        self._h = h
        self.precision = precision
        if precision == "mixed":
            st = lib().or_set_mixed(h)
            if st != 0:
                self.close()
                raise OracleError(st)

    def close(self):
        if self._h:
            lib().or_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_n(self, l):
        return lib().or_level_n(self._h, l)

    def level_k(self, l):
        n = self.level_n(l)
        sx, sy, sz = face_shapes(n)
        kx, ky, kz = np.empty(sx), np.empty(sy), np.empty(sz)
        lib().or_get_k(self._h, l, _p(kx), _p(ky), _p(kz))
        return kx, ky, kz

    def level_interval(self, l):
        """Chebyshev interval (lo, hi) of D^-1 A used on level l."""
        lo, hi = ctypes.c_double(), ctypes.c_double()
        if lib().or_level_interval(self._h, l, ctypes.byref(lo), ctypes.byref(hi)) != 0:
            raise OracleError(1)
        return lo.value, hi.value

    def level_a27(self, l):
        """27-point Galerkin operator of level l as an (N,N,N,27) array (index (dz+1)*9+(dy+1)*3+(dx+1))."""
        n = self.level_n(l)
        out = np.empty((n, n, n, 27))
        if lib().or_get_a27(self._h, l, _p(out)) != 0:
            raise OracleError(1)
        return out

    def apply(self, l, u):
        u = _f64(u)
        out = np.empty_like(u)
        lib().or_apply(self._h, l, _p(u), _p(out))
        return out

    def smooth(self, l, b, x0=None):
        b = _f64(b)
        x = np.zeros_like(b) if x0 is None else _f64(x0).copy()
        lib().or_smooth(self._h, l, _p(b), _p(x), 1 if x0 is None else 0)
        return x

    def coarse_solve(self, b):
        b = _f64(b)
        x = np.empty_like(b)
        lib().or_coarse_solve(self._h, _p(b), _p(x))
        return x

    def vcycle(self, r):
        r = _f64(r)
        z = np.empty_like(r)
        lib().or_vcycle(self._h, _p(r), _p(z))
        return z

    def solve(self, f, rtol=1e-8, max_it=200, flexible=False):
        """PCG from x0 = 0 (flexible: Polak-Ribiere beta).  Returns (x, info dict);
        raises only on argument errors."""
        f = _f64(f)
        x = np.zeros_like(f)
        its = ctypes.c_int(0)
        rr = ctypes.c_double(0)
        rt = ctypes.c_double(0)
        cits = ctypes.c_long(0)
        st = lib().or_pcg2(self._h, _p(f), _p(x), rtol, max_it, 1 if flexible else 0, ctypes.byref(its),
                           ctypes.byref(rr), ctypes.byref(rt), ctypes.byref(cits))
        if st in (1, 4):
            raise OracleError(st)
        return x, {"status": STATUS[st], "iterations": its.value, "rel_res": rr.value,
                   "rel_res_true": rt.value, "coarse_iterations": cits.value,
                   "restarts": lib().or_last_restarts(self._h)}

    def last_direction(self):
        """The CG search direction as the last solve left it (test observable)."""
        p = np.empty((self.n, self.n, self.n))
        if lib().or_last_direction(self._h, _p(p)) != 0:
            raise OracleError(1)
        return p

    def adjoint_gradient(self, phi, dl_dphi, rtol=1e-12, max_it=200):
        """Return (g_x, g_y, g_z, lambda, info): g = dL/d(ln k) on the face arrays."""
        phi, dl = _f64(phi), _f64(dl_dphi)
        n = self.n
        sx, sy, sz = face_shapes(n)
        gx, gy, gz = np.empty(sx), np.empty(sy), np.empty(sz)
        lam = np.empty((n, n, n))
        its = ctypes.c_int(0)
        st = lib().or_adjoint_gradient(self._h, _p(phi), _p(dl), _p(gx), _p(gy), _p(gz), _p(lam),
                                       rtol, max_it, ctypes.byref(its))
        if st in (1, 4):
            raise OracleError(st)
        return gx, gy, gz, lam, {"status": STATUS[st], "iterations": its.value}
