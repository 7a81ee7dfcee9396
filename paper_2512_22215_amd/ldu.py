"""Python binding of libldu.so (ctypes; argument marshalling only).

Every computation runs in the HIP library.  PyTorch provides device memory
(tensors on the GPU) and the current HIP stream; nothing here computes on the
CPU, and a missing library raises instead of falling back.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libldu.so")

LDU_OK, LDU_NOT_CONVERGED = 0, 1
LDU_ERR_ARG, LDU_ERR_ADDR, LDU_ERR_NAN, LDU_ERR_BREAKDOWN = -1, -2, -3, -4
LDU_ERR_NOMEM, LDU_ERR_HIP, LDU_ERR_STATE, LDU_ERR_LIMIT = -5, -6, -7, -8
LDU_FP64, LDU_MIXED = 0, 1
SOLVERS = {"pcg": 0, "gamg": 1, "pbicg": 2}

EXPORTED = (
    "ldu_pcg_default_opts", "ldu_gamg_default_opts", "ldu_create", "ldu_set_coeffs",
    "ldu_destroy", "ldu_amul", "ldu_tmul", "ldu_amul_f32", "ldu_residual", "pcg_solve",
    "pcg_solve_noalloc",
    "pbicg_solve", "gamg_setup", "gamg_solve", "gamg_vcycle", "gamg_level_size", "gamg_level_export",
    "ldu_level_layout", "ldu_level_downleg", "ldu_adjoint_solve", "ldu_coeff_grad",
    "ldu_assemble_pressure", "ldu_last_error",
)


# ldu_bench.h: bandwidth-ceiling kernels (measurement aids)
BENCH_EXPORTED = ("ldu_stream_read", "ldu_stream_copy", "ldu_stream_cg_update")


class LduError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ldu error {code}: {msg}")
        self.code = code


class PcgOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("precond", C.c_int), ("precision", C.c_int),
                ("max_refine", C.c_int), ("inner_max_iter", C.c_int),
                ("inner_rel_tol", C.c_double)]


class GamgOpts(C.Structure):
    _fields_ = [("rel_tol", C.c_double), ("abs_tol", C.c_double), ("max_cycles", C.c_int),
                ("n_coarsest", C.c_int), ("n_pre", C.c_int), ("n_post", C.c_int),
                ("max_levels", C.c_int), ("scale_correction", C.c_int),
                ("match_rounds", C.c_int), ("precision", C.c_int), ("max_refine", C.c_int),
                ("omega", C.c_double), ("passes", C.c_int), ("aggressive_from", C.c_int),
                ("smoother", C.c_int),
                ("gs_inner", C.c_int), ("coarsest", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("refinements", C.c_int), ("converged", C.c_int),
                ("n_levels", C.c_int), ("initial_residual", C.c_double),
                ("final_residual", C.c_double), ("level_cells", C.c_longlong * 64),
                ("level_faces", C.c_longlong * 64), ("history", C.POINTER(C.c_double)),
                ("history_len", C.c_int), ("history_count", C.c_int)]


@dataclass
class SolveStats:
    status: int
    iterations: int
    refinements: int
    converged: bool
    n_levels: int
    initial_residual: float
    final_residual: float
    level_cells: list = field(default_factory=list)
    level_faces: list = field(default_factory=list)
    history: list = field(default_factory=list)


_lib = None


def lib():
    """Load libldu.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, i = C.c_void_p, C.c_int32, C.c_int64, C.c_int
    L.ldu_pcg_default_opts.argtypes = [C.POINTER(PcgOpts)]
    L.ldu_gamg_default_opts.argtypes = [C.POINTER(GamgOpts)]
    L.ldu_create.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]
    L.ldu_set_coeffs.argtypes = [vp, vp, vp, vp, vp]
    L.ldu_destroy.argtypes = [vp]
    for f in (L.ldu_amul, L.ldu_tmul, L.ldu_amul_f32):
        f.argtypes = [vp, vp, vp, vp]
    L.ldu_residual.argtypes = [vp, vp, vp, C.POINTER(C.c_double), vp]
    L.pcg_solve.argtypes = [vp, vp, vp, C.POINTER(PcgOpts), C.POINTER(Stats), vp]
    L.pbicg_solve.argtypes = L.pcg_solve.argtypes
    L.pcg_solve_noalloc.argtypes = L.pcg_solve.argtypes
    L.gamg_setup.argtypes = [vp, C.POINTER(GamgOpts), vp]
    L.gamg_solve.argtypes = [vp, vp, vp, C.POINTER(GamgOpts), C.POINTER(Stats), vp]
    L.gamg_vcycle.argtypes = [vp, vp, vp, C.POINTER(GamgOpts), vp]
    L.gamg_level_size.argtypes = [vp, i, C.POINTER(i64), C.POINTER(i64)]
    L.gamg_level_export.argtypes = [vp, i, vp, vp, vp, vp, vp, vp, vp]
    L.ldu_level_layout.argtypes = [vp, i, C.POINTER(i), C.POINTER(i)]
    L.ldu_level_downleg.argtypes = [vp, i, C.POINTER(i), C.POINTER(i)]
    L.ldu_adjoint_solve.argtypes = [vp, vp, vp, i, vp, C.POINTER(Stats), vp]
    L.ldu_coeff_grad.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.ldu_assemble_pressure.argtypes = [vp] * 13
    L.ldu_last_error.restype = C.c_char_p
    # bandwidth-ceiling kernels of ldu_bench.h
    L.ldu_stream_read.argtypes = [vp, i64, vp, i, i, vp]
    L.ldu_stream_copy.argtypes = [vp, vp, i64, i, i, vp]
    L.ldu_stream_cg_update.argtypes = [vp, vp, vp, vp, C.c_double, i64, i, i, vp]
    for name in BENCH_EXPORTED:
        getattr(L, name).restype = C.c_int
    for name in EXPORTED:
        if name != "ldu_last_error" and name not in ("ldu_pcg_default_opts",
                                                     "ldu_gamg_default_opts"):
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc, allow_not_converged=True):
    if rc == LDU_OK or (allow_not_converged and rc == LDU_NOT_CONVERGED):
        return rc
    raise LduError(rc, lib().ldu_last_error().decode())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, device):
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype).contiguous()


def pcg_opts(**kw) -> PcgOpts:
    o = PcgOpts()
    lib().ldu_pcg_default_opts(C.byref(o))
    if "precision" in kw and isinstance(kw["precision"], str):
        kw["precision"] = LDU_MIXED if kw["precision"] == "mixed" else LDU_FP64
    for k, v in kw.items():
        setattr(o, k, v)
    return o


SMOOTHERS = {"jacobi": 0, "gs2": 1}
COARSEST = {"diag": 0, "dic": 1}


def gamg_opts(**kw) -> GamgOpts:
    o = GamgOpts()
    lib().ldu_gamg_default_opts(C.byref(o))
    if "precision" in kw and isinstance(kw["precision"], str):
        kw["precision"] = LDU_MIXED if kw["precision"] == "mixed" else LDU_FP64
    if isinstance(kw.get("smoother"), str):
        kw["smoother"] = SMOOTHERS[kw["smoother"]]
    if isinstance(kw.get("coarsest"), str):
        kw["coarsest"] = COARSEST[kw["coarsest"]]
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stats_out(rc, s: Stats, hist_buf) -> SolveStats:
    nl = max(s.n_levels, 0)
    return SolveStats(rc, s.iterations, s.refinements, bool(s.converged), s.n_levels,
                      s.initial_residual, s.final_residual,
                      list(s.level_cells[:nl]), list(s.level_faces[:nl]),
                      list(hist_buf[: s.history_count]) if hist_buf is not None else [])


class LduMatrix:
    """An LDU matrix resident on the GPU (paper Sec. 2.1 storage)."""

    def __init__(self, n_cells, owner, neighbour, diag, upper, lower, device="cuda"):
        self.device = torch.device(device)
        self.n = int(n_cells)
        self.owner = _dev(owner, torch.int32, self.device)
        self.neighbour = _dev(neighbour, torch.int32, self.device)
        self.nf = int(self.owner.numel())
        d = _dev(diag, torch.float64, self.device)
        u = _dev(upper, torch.float64, self.device)
        l = _dev(lower, torch.float64, self.device)
        h = C.c_void_p()
        _check(lib().ldu_create(self.n, self.nf, _ptr(self.owner), _ptr(self.neighbour),
                                _ptr(d), _ptr(u), _ptr(l), _stream(), C.byref(h)), False)
        self._h = h
        # bumped by every call that replaces the coefficients
        self.coeff_version = 0

    @classmethod
    def from_case(cls, case, device="cuda"):
        return cls(case.n_cells, case.owner, case.neighbour, case.diag, case.upper,
                   case.lower, device)

    def close(self):
        h, self._h = getattr(self, "_h", None), None
        if h and h.value and _lib is not None:
            _lib.ldu_destroy(h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def _vec(self, x, dtype=torch.float64):
        return _dev(x, dtype, self.device)

    def _sized(self, x, count, what):
        t = self._vec(x)
        if t.numel() != count:
            raise ValueError(f"{what}: {t.numel()} values, expected {count}")
        return t

    def set_coeffs(self, diag, upper, lower):
        d, u, l = (self._vec(v) for v in (diag, upper, lower))
        self.coeff_version += 1
        _check(lib().ldu_set_coeffs(self._h, _ptr(d), _ptr(u), _ptr(l), _stream()), False)

    def amul(self, x, out=None):
        x = self._vec(x)
        y = torch.empty_like(x) if out is None else out
        _check(lib().ldu_amul(self._h, _ptr(x), _ptr(y), _stream()), False)
        return y

    def tmul(self, x, out=None):
        x = self._vec(x)
        y = torch.empty_like(x) if out is None else out
        _check(lib().ldu_tmul(self._h, _ptr(x), _ptr(y), _stream()), False)
        return y

    def amul_f32(self, x, out=None):
        x = self._vec(x, torch.float32)
        y = torch.empty_like(x) if out is None else out
        _check(lib().ldu_amul_f32(self._h, _ptr(x), _ptr(y), _stream()), False)
        return y

    def residual(self, b, x):
        out = C.c_double()
        b, x = self._vec(b), self._vec(x)
        _check(lib().ldu_residual(self._h, _ptr(b), _ptr(x), C.byref(out), _stream()), False)
        return out.value

    def _solve(self, fn, b, x0, opts, history):
        b = self._vec(b)
        x = torch.zeros_like(b) if x0 is None else self._vec(x0).clone()
        st = Stats()
        buf = None
        if history:
            buf = (C.c_double * history)()
            st.history = C.cast(buf, C.POINTER(C.c_double))
            st.history_len = history
        rc = fn(self._h, _ptr(b), _ptr(x), C.byref(opts), C.byref(st), _stream())
        _check(rc)
        return x, _stats_out(rc, st, buf)

    def pcg(self, b, x0=None, history=0, **kw):
        return self._solve(lib().pcg_solve, b, x0, pcg_opts(**kw), history)

    def pcg_noalloc(self, b, x0=None, history=0, **kw):
        """pcg_solve_noalloc: diagonal (or no) preconditioner, FP64, with the
        library's static scratch instead of device allocations."""
        return self._solve(lib().pcg_solve_noalloc, b, x0, pcg_opts(**kw), history)

    def gamg(self, b, x0=None, history=0, **kw):
        return self._solve(lib().gamg_solve, b, x0, gamg_opts(**kw), history)

    def pbicg(self, b, x0=None, history=0, **kw):
        """Preconditioned bi-conjugate gradients (non-symmetric A)."""
        return self._solve(lib().pbicg_solve, b, x0, pcg_opts(**kw), history)

    def gamg_setup(self, **kw):
        o = gamg_opts(**kw)
        _check(lib().gamg_setup(self._h, C.byref(o), _stream()), False)

    def vcycle(self, r, **kw):
        r = self._vec(r)
        e = torch.empty_like(r)
        o = gamg_opts(**kw)
        _check(lib().gamg_vcycle(self._h, _ptr(r), _ptr(e), C.byref(o), _stream()), False)
        return e

    def n_levels(self):
        l = 0
        while True:
            n = C.c_int64()
            if lib().gamg_level_size(self._h, l, C.byref(n), None) != LDU_OK:
                return l
            l += 1

    def level(self, l):
        n, nf = C.c_int64(), C.c_int64()
        _check(lib().gamg_level_size(self._h, l, C.byref(n), C.byref(nf)), False)
        n, nf = n.value, nf.value
        dv = self.device
        out = {"n": n, "nf": nf,
               "agg": torch.full((n,), -1, dtype=torch.int32, device=dv),
               "owner": torch.empty(nf, dtype=torch.int32, device=dv),
               "neighbour": torch.empty(nf, dtype=torch.int32, device=dv),
               "diag": torch.empty(n, dtype=torch.float64, device=dv),
               "upper": torch.empty(nf, dtype=torch.float64, device=dv),
               "lower": torch.empty(nf, dtype=torch.float64, device=dv)}
        _check(lib().gamg_level_export(self._h, l, _ptr(out["agg"]), _ptr(out["owner"]),
                                       _ptr(out["neighbour"]), _ptr(out["diag"]),
                                       _ptr(out["upper"]), _ptr(out["lower"]), _stream()),
               False)
        return out

    def layout(self, l=0):
        """Storage of level l in the product kernels: {"compressed", "col16"}."""
        cmp_, c16 = C.c_int(), C.c_int()
        _check(lib().ldu_level_layout(self._h, l, C.byref(cmp_), C.byref(c16)), False)
        return {"compressed": bool(cmp_.value), "col16": bool(c16.value)}

    def downleg(self, l):
        """Form of level l's one-pass down leg: ("none" | "r_compressed" |
        "r_csr" | "scaled_slices", lanes per row of a CSR R)."""
        form, lanes = C.c_int(), C.c_int()
        _check(lib().ldu_level_downleg(self._h, l, C.byref(form), C.byref(lanes)), False)
        names = {0: "none", 1: "r_compressed", 2: "r_csr", 3: "scaled_slices"}
        return names[form.value], lanes.value

    def adjoint(self, g, use_gamg=False, x0=None, history=0, solver=None, **kw):
        """A^T lambda = g; solver "pcg" (default), "gamg" (or use_gamg=True) or
        "pbicg"."""
        g = self._vec(g)
        lam = torch.zeros_like(g) if x0 is None else self._vec(x0).clone()
        solver = solver or ("gamg" if use_gamg else "pcg")
        opts = gamg_opts(**kw) if solver == "gamg" else pcg_opts(**kw)
        st = Stats()
        buf = None
        if history:
            buf = (C.c_double * history)()
            st.history = C.cast(buf, C.POINTER(C.c_double))
            st.history_len = history
        rc = lib().ldu_adjoint_solve(self._h, _ptr(g), _ptr(lam), SOLVERS[solver],
                                     C.cast(C.pointer(opts), C.c_void_p), C.byref(st),
                                     _stream())
        _check(rc)
        return lam, _stats_out(rc, st, buf)

    def assemble_pressure(self, gamma, weights, mag_sf, delta, diag_bc=None, phi=None,
                          b_bc=None, out_coeffs=False):
        """Assemble the pressure equation on this mesh (replaces the
        coefficients).  Returns b (or None without phi), plus (diag, upper,
        lower) copies when out_coeffs."""
        n, nf = self.n, self.nf
        gamma = self._sized(gamma, n, "gamma")
        weights = self._sized(weights, nf, "weights")
        mag_sf = self._sized(mag_sf, nf, "mag_sf")
        delta = self._sized(delta, nf, "delta")
        diag_bc = None if diag_bc is None else self._sized(diag_bc, n, "diag_bc")
        b_bc = None if b_bc is None else self._sized(b_bc, n, "b_bc")
        phi = None if phi is None else self._sized(phi, nf, "phi")
        b = None if phi is None else torch.empty(self.n, dtype=torch.float64,
                                                 device=self.device)
        outs = [None, None, None]
        if out_coeffs:
            outs = [torch.empty(k, dtype=torch.float64, device=self.device)
                    for k in (self.n, self.nf, self.nf)]
        p = lambda t: None if t is None else _ptr(t)
        self.coeff_version += 1
        _check(lib().ldu_assemble_pressure(self._h, p(gamma), p(weights), p(mag_sf), p(delta),
                                           p(diag_bc), p(phi), p(b_bc), p(b), p(outs[0]),
                                           p(outs[1]), p(outs[2]), _stream()), False)
        return (b, tuple(outs)) if out_coeffs else b

    def coeff_grad(self, lam, x):
        lam, x = self._vec(lam), self._vec(x)
        gd = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gu = torch.empty(self.nf, dtype=torch.float64, device=self.device)
        gl = torch.empty(self.nf, dtype=torch.float64, device=self.device)
        _check(lib().ldu_coeff_grad(self._h, _ptr(lam), _ptr(x), _ptr(gd), _ptr(gu),
                                    _ptr(gl), _stream()), False)
        return gd, gu, gl
