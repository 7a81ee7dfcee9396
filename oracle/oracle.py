"""ctypes binding of the C oracle (test infrastructure only).

Builds oracle/libldu_oracle.so with gcc on first use when it is missing.
Every function takes and returns numpy arrays; nothing here touches a GPU.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ldu_oracle.c")
# ORACLE_SANITIZE=1 selects a build with AddressSanitizer and
# UndefinedBehaviorSanitizer (every report aborts); the process must then
# preload the ASan runtime (see tests/test_oracle_sanitized.py)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "libldu_oracle_san.so" if _SANITIZE else "libldu_oracle.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_ADDR, ERR_NAN, ERR_BREAKDOWN = -1, -2, -3, -4


def build(force: bool = False) -> str:
    """Compile the oracle (plain C, no FMA contraction, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(
            os.path.getmtime(_SRC),
            os.path.getmtime(os.path.join(_HERE, "ldu_oracle.h"))):
        tmp = _LIB + ".tmp"
        san = (["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                "-fno-sanitize-recover=all"] if _SANITIZE else [])
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
             "-Wall", "-fPIC", "-shared"] + san + ["-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None

_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


def _opt(ptr_t):
    """ndpointer that also accepts None."""
    class _P(ptr_t):
        @classmethod
        def from_param(cls, obj):
            if obj is None:
                return None
            return ptr_t.from_param(obj)
    return _P


_f64o = _opt(_f64p)
_i32o = _opt(_i32p)


def lib():
    global _lib
    if _lib is not None:
        return _lib
    L = C.CDLL(build())
    i32, i64, d, vp = C.c_int32, C.c_int64, C.c_double, C.c_void_p
    ip = C.POINTER(C.c_int)
    dp = C.POINTER(C.c_double)
    L.orc_validate.argtypes = [i32, i64, _i32p, _i32p, _f64o, _f64o, _f64o]
    L.orc_amul.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]
    L.orc_tmul.argtypes = L.orc_amul.argtypes
    L.orc_amul_f32.argtypes = [i32, i64, _i32p, _i32p, _f32p, _f32p, _f32p, _f32p, _f32p]
    L.orc_pcg.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p,
                          d, C.c_int, C.c_int, C.c_int, ip, _f64o, dp]
    L.orc_pbicg.argtypes = L.orc_pcg.argtypes
    L.orc_assemble_pressure.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p,
                                        _f64o, _f64o, _f64o, _f64p, _f64p, _f64p, _f64o]
    L.orc_pcg_mixed.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p,
                                _f64p, d, C.c_int, d, C.c_int, C.c_int, ip, ip, _f64o, dp]
    L.orc_gamg_build.restype = vp
    L.orc_gamg_build.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p,
                                 C.c_int, C.c_int, C.c_int]
    L.orc_gamg_build2.restype = vp
    L.orc_gamg_build2.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p,
                                  C.c_int, C.c_int, C.c_int, C.c_int]
    L.orc_gamg_build3.restype = vp
    L.orc_gamg_build3.argtypes = L.orc_gamg_build2.argtypes + [C.c_int]
    L.orc_gamg_free.argtypes = [vp]
    L.orc_gamg_set_cycle.argtypes = [vp, C.c_int, C.c_int, C.c_int]
    L.orc_gs2_sweep.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                C.c_int, C.c_int, C.c_int]
    L.orc_gs2_sweep32.argtypes = [i32, i64, _i32p, _i32p, _f32p, _f32p, _f32p, _f32p,
                                  _f32p, C.c_int, C.c_int, C.c_int]
    L.orc_dic.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p, _f64o, _f64o, _f64o]
    L.orc_gamg_set_values.argtypes = [vp, _f64p, _f64p, _f64p]
    L.orc_gamg_nlevels.argtypes = [vp]
    L.orc_gamg_level_size.argtypes = [vp, C.c_int, C.POINTER(i64), C.POINTER(i64)]
    L.orc_gamg_level_export.argtypes = [vp, C.c_int, _i32o, _i32o, _i32o, _f64o,
                                        _f64o, _f64o]
    L.orc_gamg_level_match.argtypes = [vp, C.c_int, _i32o, _i32o]
    L.orc_gamg_vcycle.argtypes = [vp, _f64p, _f64p, C.c_int, C.c_int, d, C.c_int,
                                  C.c_int]
    L.orc_gamg_vcycle32.argtypes = [vp, _f32p, _f32p, C.c_int, C.c_int, d, C.c_int,
                                    C.c_int]
    L.orc_gamg_solve.argtypes = [vp, _f64p, _f64p, d, C.c_int, C.c_int, C.c_int, d,
                                 C.c_int, C.c_int, ip, _f64o, dp]
    L.orc_pcg_gamg.argtypes = [vp, _f64p, _f64p, d, C.c_int, C.c_int, C.c_int, d,
                               C.c_int, ip, _f64o, dp]
    L.orc_pcg_gamg_mixed.argtypes = [vp, _f64p, _f64p, d, C.c_int, d, C.c_int, C.c_int,
                                     C.c_int, d, C.c_int, ip, ip, _f64o, dp]
    L.orc_gamg_mixed.argtypes = [vp, _f64p, _f64p, d, C.c_int, C.c_int, C.c_int, d,
                                 C.c_int, C.c_int, ip, _f64o, dp]
    L.orc_coeff_grad.argtypes = [i32, i64, _i32p, _i32p, _f64p, _f64p, _f64p,
                                 _f64p, _f64p]
    _lib = L
    return L


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Ldu:
    """An LDU matrix as held by the oracle (plain numpy arrays)."""

    def __init__(self, n, owner, neighbour, diag, upper, lower):
        self.n = int(n)
        self.own = _c(owner, np.int32)
        self.nb = _c(neighbour, np.int32)
        self.diag = _c(diag, np.float64)
        self.upper = _c(upper, np.float64)
        self.lower = _c(lower, np.float64)
        self.nf = int(self.own.shape[0])

    @classmethod
    def from_case(cls, case):
        return cls(case.n_cells, case.owner, case.neighbour, case.diag,
                   case.upper, case.lower)

    def args(self):
        return (self.n, self.nf, self.own, self.nb, self.diag, self.upper,
                self.lower)


def validate(n, owner, neighbour, diag=None, upper=None, lower=None):
    return lib().orc_validate(
        int(n), int(len(owner)), _c(owner, np.int32), _c(neighbour, np.int32),
        None if diag is None else _c(diag, np.float64),
        None if upper is None else _c(upper, np.float64),
        None if lower is None else _c(lower, np.float64))


def amul(A: Ldu, x):
    y = np.empty(A.n)
    lib().orc_amul(*A.args(), _c(x, np.float64), y)
    return y


def tmul(A: Ldu, x):
    y = np.empty(A.n)
    lib().orc_tmul(*A.args(), _c(x, np.float64), y)
    return y


def amul_f32(A: Ldu, x):
    y = np.empty(A.n, np.float32)
    lib().orc_amul_f32(A.n, A.nf, A.own, A.nb, A.diag.astype(np.float32),
                       A.upper.astype(np.float32), A.lower.astype(np.float32),
                       _c(x, np.float32), y)
    return y


@dataclass
class SolveResult:
    status: int
    x: np.ndarray
    iterations: int
    history: np.ndarray
    true_residual: float
    inner_iterations: int = 0


def pcg(A: Ldu, b, x0=None, tol=1e-8, max_iter=10000, precond=True,
        transpose=False):
    x = np.zeros(A.n) if x0 is None else _c(x0, np.float64).copy()
    hist = np.zeros(max_iter + 2)
    it = C.c_int(0)
    tr = C.c_double(0.0)
    st = lib().orc_pcg(*A.args(), _c(b, np.float64), x, float(tol),
                       int(max_iter), int(bool(precond)), int(bool(transpose)),
                       C.byref(it), hist, C.byref(tr))
    return SolveResult(st, x, it.value, hist[: it.value + 1].copy(), tr.value)


def pbicg(A: Ldu, b, x0=None, tol=1e-8, max_iter=10000, precond=True,
          transpose=False):
    """Preconditioned bi-conjugate gradients (non-symmetric A)."""
    x = np.zeros(A.n) if x0 is None else _c(x0, np.float64).copy()
    hist = np.zeros(max_iter + 2)
    it = C.c_int(0)
    tr = C.c_double(0.0)
    st = lib().orc_pbicg(*A.args(), _c(b, np.float64), x, float(tol),
                         int(max_iter), int(bool(precond)), int(bool(transpose)),
                         C.byref(it), hist, C.byref(tr))
    return SolveResult(st, x, it.value, hist[: it.value + 1].copy(), tr.value)


def pcg_mixed(A: Ldu, b, x0=None, tol=1e-8, max_refine=50, inner_tol=1e-4,
              inner_max_iter=1000, transpose=False):
    x = np.zeros(A.n) if x0 is None else _c(x0, np.float64).copy()
    hist = np.zeros(max_refine + 2)
    k = C.c_int(0)
    inner = C.c_int(0)
    tr = C.c_double(0.0)
    st = lib().orc_pcg_mixed(*A.args(), _c(b, np.float64), x, float(tol),
                             int(max_refine), float(inner_tol),
                             int(inner_max_iter), int(bool(transpose)),
                             C.byref(k), C.byref(inner), hist, C.byref(tr))
    return SolveResult(st, x, k.value, hist[: k.value + 1].copy(), tr.value,
                       inner.value)


@dataclass
class Level:
    n: int
    nf: int
    agg: np.ndarray | None
    owner: np.ndarray
    neighbour: np.ndarray
    diag: np.ndarray
    upper: np.ndarray
    lower: np.ndarray
    partner: np.ndarray | None = None
    join: np.ndarray | None = None


class Gamg:
    """Oracle GAMG hierarchy (built once; values and structure fixed)."""

    SMOOTHERS = {"jacobi": 0, "gs2": 1}
    COARSEST = {"diag": 0, "dic": 1}

    def __init__(self, A: Ldu, n_coarsest=50, max_levels=50, match_rounds=16,
                 passes=1, smoother="jacobi", gs_inner=1, coarsest="diag",
                 aggressive_from=0):
        """smoother: "jacobi" (damped Jacobi / Richardson) or "gs2" (two-stage
        Gauss-Seidel with gs_inner inner steps); coarsest: the coarsest-level
        CG preconditioner, "diag" or "dic"."""
        self.A = A
        self._h = lib().orc_gamg_build3(*A.args(), int(n_coarsest),
                                        int(max_levels), int(match_rounds),
                                        int(passes), int(aggressive_from))
        rc = lib().orc_gamg_set_cycle(self._h, self.SMOOTHERS[smoother], int(gs_inner),
                                      self.COARSEST[coarsest])
        if rc != OK:
            raise ValueError("invalid cycle options")

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _lib is not None:
            _lib.orc_gamg_free(h)

    def set_values(self, diag, upper, lower):
        """New fine-level coefficients; aggregation kept, Galerkin redone."""
        lib().orc_gamg_set_values(self._h, _c(diag, np.float64),
                                  _c(upper, np.float64), _c(lower, np.float64))

    @property
    def n_levels(self):
        return lib().orc_gamg_nlevels(self._h)

    def level(self, l) -> Level:
        n = C.c_int64()
        nf = C.c_int64()
        lib().orc_gamg_level_size(self._h, l, C.byref(n), C.byref(nf))
        n, nf = n.value, nf.value
        coarsest = l == self.n_levels - 1
        agg = None if coarsest else np.empty(n, np.int32)
        own = np.empty(nf, np.int32)
        nb = np.empty(nf, np.int32)
        d = np.empty(n)
        u = np.empty(nf)
        lo = np.empty(nf)
        lib().orc_gamg_level_export(self._h, l, agg, own, nb, d, u, lo)
        partner = join = None
        if not coarsest:
            partner = np.empty(n, np.int32)
            join = np.empty(n, np.int32)
            lib().orc_gamg_level_match(self._h, l, partner, join)
        return Level(n, nf, agg, own, nb, d, u, lo, partner, join)

    def vcycle(self, r, n_pre=2, n_post=2, omega=0.75, scale=True,
               transpose=False):
        e = np.zeros(self.A.n)
        lib().orc_gamg_vcycle(self._h, _c(r, np.float64), e, int(n_pre),
                              int(n_post), float(omega), int(bool(scale)),
                              int(bool(transpose)))
        return e

    def vcycle_f32(self, r, n_pre=2, n_post=2, omega=0.75, scale=True,
                   transpose=False):
        """The FP32 V-cycle of the mixed-precision solvers."""
        e = np.zeros(self.A.n, np.float32)
        lib().orc_gamg_vcycle32(self._h, _c(r, np.float32), e, int(n_pre),
                                int(n_post), float(omega), int(bool(scale)),
                                int(bool(transpose)))
        return e

    def solve(self, b, x0=None, tol=1e-8, max_cycles=200, n_pre=2, n_post=2,
              omega=0.75, scale=True, transpose=False):
        x = np.zeros(self.A.n) if x0 is None else _c(x0, np.float64).copy()
        hist = np.zeros(max_cycles + 2)
        k = C.c_int(0)
        tr = C.c_double(0.0)
        st = lib().orc_gamg_solve(self._h, _c(b, np.float64), x, float(tol),
                                  int(max_cycles), int(n_pre), int(n_post),
                                  float(omega), int(bool(scale)),
                                  int(bool(transpose)), C.byref(k), hist,
                                  C.byref(tr))
        return SolveResult(st, x, k.value, hist[: k.value + 1].copy(), tr.value)

    def pcg(self, b, x0=None, tol=1e-8, max_iter=10000, n_pre=2, n_post=2,
            omega=0.75, transpose=False):
        """CG preconditioned by one V-cycle (correction scaling off)."""
        x = np.zeros(self.A.n) if x0 is None else _c(x0, np.float64).copy()
        hist = np.zeros(max_iter + 2)
        k = C.c_int(0)
        tr = C.c_double(0.0)
        st = lib().orc_pcg_gamg(self._h, _c(b, np.float64), x, float(tol),
                                int(max_iter), int(n_pre), int(n_post),
                                float(omega), int(bool(transpose)), C.byref(k),
                                hist, C.byref(tr))
        return SolveResult(st, x, k.value, hist[: k.value + 1].copy(), tr.value)

    def pcg_mixed(self, b, x0=None, tol=1e-8, max_refine=50, inner_tol=1e-4,
                  inner_max_iter=1000, n_pre=2, n_post=2, omega=0.75,
                  transpose=False):
        """FP64 refinement around FP32 CG preconditioned by an FP32 V-cycle."""
        x = np.zeros(self.A.n) if x0 is None else _c(x0, np.float64).copy()
        hist = np.zeros(max_refine + 2)
        k = C.c_int(0)
        inner = C.c_int(0)
        tr = C.c_double(0.0)
        st = lib().orc_pcg_gamg_mixed(self._h, _c(b, np.float64), x, float(tol),
                                      int(max_refine), float(inner_tol),
                                      int(inner_max_iter), int(n_pre), int(n_post),
                                      float(omega), int(bool(transpose)),
                                      C.byref(k), C.byref(inner), hist, C.byref(tr))
        return SolveResult(st, x, k.value, hist[: k.value + 1].copy(), tr.value,
                           inner.value)

    def solve_mixed(self, b, x0=None, tol=1e-8, max_refine=200, n_pre=2,
                    n_post=2, omega=0.75, scale=True, transpose=False):
        x = np.zeros(self.A.n) if x0 is None else _c(x0, np.float64).copy()
        hist = np.zeros(max_refine + 2)
        k = C.c_int(0)
        tr = C.c_double(0.0)
        st = lib().orc_gamg_mixed(self._h, _c(b, np.float64), x, float(tol),
                                  int(max_refine), int(n_pre), int(n_post),
                                  float(omega), int(bool(scale)),
                                  int(bool(transpose)), C.byref(k), hist,
                                  C.byref(tr))
        return SolveResult(st, x, k.value, hist[: k.value + 1].copy(), tr.value)


def coeff_grad(A: Ldu, lam, x):
    gd = np.empty(A.n)
    gu = np.empty(A.nf)
    gl = np.empty(A.nf)
    lib().orc_coeff_grad(A.n, A.nf, A.own, A.nb, _c(lam, np.float64),
                         _c(x, np.float64), gd, gu, gl)
    return gd, gu, gl


def gs2_sweep(A: Ldu, r, e=None, backward=False, inner=1):
    """One two-stage Gauss-Seidel sweep on A e = r (from e = 0 when e is None)."""
    out = np.zeros(A.n) if e is None else _c(e, np.float64).copy()
    lib().orc_gs2_sweep(*A.args(), _c(r, np.float64), out, int(e is None),
                        int(bool(backward)), int(inner))
    return out


def gs2_sweep_f32(A: Ldu, r, e=None, backward=False, inner=1):
    """The FP32 two-stage Gauss-Seidel sweep of the mixed-precision V-cycle
    (coefficients and vectors rounded to FP32)."""
    out = np.zeros(A.n, np.float32) if e is None else _c(e, np.float32).copy()
    lib().orc_gs2_sweep32(A.n, A.nf, A.own, A.nb, A.diag.astype(np.float32),
                          A.upper.astype(np.float32), A.lower.astype(np.float32),
                          _c(r, np.float32), out, int(e is None), int(bool(backward)),
                          int(inner))
    return out


def dic(A: Ldu, r=None):
    """DIC pivots Dt, usability flag, and z = M^-1 r when r is given."""
    dt = np.empty(A.n)
    z = None if r is None else np.empty(A.n)
    ok = lib().orc_dic(*A.args(), dt, None if r is None else _c(r, np.float64), z)
    return dt, bool(ok), z


def assemble_pressure(n, owner, neighbour, gamma, weights, mag_sf, delta, diag_bc=None,
                      phi=None, b_bc=None):
    """Pressure-equation assembly: returns (diag, upper, lower, b or None)."""
    own = _c(owner, np.int32)
    nb = _c(neighbour, np.int32)
    nf = own.size
    diag = np.empty(n)
    up = np.empty(nf)
    lo = np.empty(nf)
    b = None if phi is None else np.empty(n)
    opt = lambda a: None if a is None else _c(a, np.float64)
    lib().orc_assemble_pressure(int(n), int(nf), own, nb, _c(gamma, np.float64),
                                _c(weights, np.float64), _c(mag_sf, np.float64),
                                _c(delta, np.float64), opt(diag_bc), opt(phi), opt(b_bc),
                                diag, up, lo, b)
    return diag, up, lo, b
