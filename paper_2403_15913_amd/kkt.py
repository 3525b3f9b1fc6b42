"""Python binding of libkkt (include/kkt.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; this module only
converts NumPy index arrays and torch device tensors into the pointers the C
ABI takes. It raises if the library has not been built -- there is no
fallback path.

Functions carry the C names (``kkt_symbolic_analyze``, ``kkt_refactor``,
``kkt_solve``, ``kkt_cg_schur`` ...); ``Symbolic`` and ``Factor`` wrap the
handles for convenience.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkkt.so")

KKT_OK = 0
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "PATTERN", 3: "STATE", 4: "NOT_SPD", 5: "NONFINITE",
                6: "NOT_CONVERGED", 7: "BREAKDOWN", 8: "OOM", 9: "BUDGET", 10: "DEVICE"}
ORDER_AUTO, ORDER_NATURAL, ORDER_ND = 0, 1, 2
SCHEDULE_LEVELS, SCHEDULE_QUEUE = 0, 1


class KKTError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Options(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("nd_leaf", C.c_int32), ("max_super", C.c_int32),
                ("relax_small", C.c_int32), ("relax_frac", C.c_double), ("front_lds_max", C.c_int32)]


class SymbolicStats(C.Structure):
    _fields_ = [("n", C.c_int32), ("m", C.c_int32), ("nsuper", C.c_int32), ("levels", C.c_int32),
                ("max_rows", C.c_int32), ("max_cols", C.c_int32), ("nnz_k", C.c_int64), ("nnz_l", C.c_int64),
                ("nnz_l_exact", C.c_int64), ("n_pairs", C.c_int64), ("flops", C.c_double),
                ("flops_exact", C.c_double), ("analyze_seconds", C.c_double), ("large_fronts", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RefineOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("tol", C.c_double)]


class SolveInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("eta", C.c_double), ("omega", C.c_double),
                ("relres", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("eta_tol", C.c_double)]


class CgInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("rel_res", C.c_double), ("eta", C.c_double),
                ("eta_stop", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class InertiaOpts(C.Structure):
    _fields_ = [("delta_first", C.c_double), ("delta_min", C.c_double), ("delta_max", C.c_double),
                ("kappa_minus", C.c_double), ("kappa_plus", C.c_double), ("kappa_plus_first", C.c_double)]


class InertiaInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("trials", C.c_int32), ("delta", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class AugInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("eta", C.c_double), ("omega", C.c_double),
                ("inner_iters", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class IpmOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxit", C.c_int32), ("sigma", C.c_double), ("tau_min", C.c_double)]


class IpmInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int32), ("err", C.c_double), ("gap", C.c_double),
                ("r1", C.c_double), ("r4", C.c_double), ("max_delta", C.c_double), ("aug_corrections", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FactorInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("bad_col", C.c_int32)]


PHASES = ["assemble", "factor", "fwd", "bwd", "residual", "permute", "cg", "control"]


class Timing(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int32 * 8)]

    def as_dict(self):
        return {p: dict(ms=self.ms[i], launches=self.launches[i]) for i, p in enumerate(PHASES)}


# Names and signatures of every exported entry point (checked by the tests
# against include/*.h).
P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
SIGNATURES = {
    "kkt_options_default": (None, [P]),
    "kkt_status_string": (C.c_char_p, [I32]),
    "kkt_last_error": (C.c_char_p, []),
    "kkt_symbolic_analyze": (I32, [I32, I32, P, P, P, P, P, P]),
    "kkt_symbolic_get_stats": (I32, [P, P]),
    "kkt_symbolic_get_perm": (I32, [P, P]),
    "kkt_symbolic_get_supernodes": (I32, [P, P, P, P]),
    "kkt_symbolic_destroy": (None, [P]),
    "kkt_factor_create": (I32, [P, P]),
    "kkt_factor_destroy": (None, [P]),
    "kkt_refactor": (I32, [P, P, P, P, P, D, P]),
    "kkt_status_sync": (I32, [P, P]),
    "kkt_inertia_opts_default": (None, [P]),
    "kkt_refactor_inertia": (I32, [P, P, P, P, P, D, P, P, P]),
    "kkt_solve_augmented": (I32, [P, P, P, P, P, P, P, P, P, P]),
    "kkt_solve": (I32, [P, P, P, P, P, P]),
    "kkt_solve_noalloc": (I32, [P, P, P, P, P, P]),
    "kkt_cg_opts_default": (None, [P]),
    "kkt_cg_schur": (I32, [P, P, P, P, P, P, P, P]),
    "kkt_matvec": (I32, [P, P, P, P]),
    "kkt_factor_set_equality_rows": (I32, [P, P, I32]),
    "kkt_factor_keep_augmented": (I32, [P, I32]),
    "kkt_ipm_opts_default": (None, [P]),
    "kkt_ipm_qp": (I32, [P, P, P, P, P, P, P, P, P, P, P]),
    "kkt_factor_set_timing": (I32, [P, I32]),
    "kkt_factor_read_timing": (I32, [P, P]),
    "kkt_factor_set_schedule": (I32, [P, I32]),
    "kkt_factor_set_update_split": (I32, [P, I32, I32]),
    "kkt_factor_set_small_fronts": (I32, [P, I32]),
    "kkt_batch_create": (I32, [I32, P, P]),
    "kkt_batch_destroy": (None, [P]),
    "kkt_batch_offsets": (I32, [P, P, P, P, P]),
    "kkt_batch_refactor": (I32, [P, P, P, P, P, P]),
    "kkt_batch_solve": (I32, [P, P, P, P, P, P]),
    "kkt_batch_status": (I32, [P, P, P]),
    "kkt_batch_set_timing": (I32, [P, I32]),
    "kkt_batch_read_timing": (I32, [P, P]),
    "kkt_batch_set_schedule": (I32, [P, I32]),
    "kkt_batch_set_update_split": (I32, [P, I32, I32]),
    "kkt_batch_set_small_fronts": (I32, [P, I32]),
    "kkt_batch_capture": (I32, [P, P, P, P, P, P, P, P, I32]),
    "kkt_batch_replay": (I32, [P, P, P]),
    "kkt_stagewise_create": (I32, [I32, P, P, P, P]),
    "kkt_stagewise_destroy": (None, [P]),
    "kkt_stagewise_refactor": (I32, [P, P, P, P, P, P]),
    "kkt_stagewise_status": (I32, [P, P, P]),
    "kkt_stagewise_solve": (I32, [P, P, P, P, P, P]),
    "kkt_stagewise_set_timing": (I32, [P, I32]),
    "kkt_stagewise_read_timing": (I32, [P, P]),
    "kkt_server_opts_default": (None, [P]),
    "kkt_server_create": (I32, [P, P]),
    "kkt_server_register": (I32, [P, P, P]),
    "kkt_server_submit": (I32, [P, I32, P, P, P, P, P, P, P, P]),
    "kkt_server_wait": (I32, [P, I64, P, P]),
    "kkt_server_get_stats": (I32, [P, P]),
    "kkt_server_reset_stats": (I32, [P]),
    "kkt_server_destroy": (None, [P]),
}

_lib = None


def lib() -> C.CDLL:
    """Load libkkt.so (built by paper_2403_15913_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2403_15913_amd.build")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _err(st: int):
    if st != KKT_OK:
        raise KKTError(st, lib().kkt_last_error().decode())


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr_np(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    """Device pointer of a torch tensor (float64, contiguous, on the GPU), or None."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous GPU tensor")
    import torch
    if t.dtype != torch.float64:
        raise ValueError("expected float64")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# functions with the C names
# ---------------------------------------------------------------------------

def kkt_options_default() -> Options:
    o = Options()
    lib().kkt_options_default(C.byref(o))
    return o


def kkt_symbolic_analyze(n, m, w_rowptr, w_colind, j_rowptr, j_colind, opt: Options | None = None):
    wr, wc, jr, jc = _i32(w_rowptr), _i32(w_colind), _i32(j_rowptr), _i32(j_colind)
    h = C.c_void_p()
    st = lib().kkt_symbolic_analyze(n, m, _ptr_np(wr), _ptr_np(wc), _ptr_np(jr), _ptr_np(jc),
                                    C.byref(opt) if opt is not None else None, C.byref(h))
    _err(st)
    return h


def kkt_symbolic_get_stats(h) -> dict:
    s = SymbolicStats()
    _err(lib().kkt_symbolic_get_stats(h, C.byref(s)))
    return s.as_dict()


def kkt_symbolic_get_perm(h, n: int) -> np.ndarray:
    out = np.empty(n, dtype=np.int32)
    _err(lib().kkt_symbolic_get_perm(h, _ptr_np(out)))
    return out


def kkt_symbolic_get_supernodes(h, nsuper: int):
    cp = np.empty(nsuper + 1, dtype=np.int32)
    par = np.empty(nsuper, dtype=np.int32)
    nr = np.empty(nsuper, dtype=np.int32)
    _err(lib().kkt_symbolic_get_supernodes(h, _ptr_np(cp), _ptr_np(par), _ptr_np(nr)))
    return cp, par, nr


def kkt_symbolic_destroy(h):
    lib().kkt_symbolic_destroy(h)


def kkt_factor_create(sym_h):
    h = C.c_void_p()
    _err(lib().kkt_factor_create(sym_h, C.byref(h)))
    return h


def kkt_factor_destroy(h):
    lib().kkt_factor_destroy(h)


def kkt_refactor(h, w_vals, j_vals, sigma_x, sigma_s=None, gamma: float = 0.0, stream=None):
    _err(lib().kkt_refactor(h, _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x), _dptr(sigma_s), float(gamma),
                            _stream(stream)))


def kkt_inertia_opts_default() -> InertiaOpts:
    o = InertiaOpts()
    lib().kkt_inertia_opts_default(C.byref(o))
    return o


def kkt_refactor_inertia(h, w_vals, j_vals, sigma_x, sigma_s=None, gamma: float = 0.0, opts: InertiaOpts | None = None,
                         stream=None) -> dict:
    ii = InertiaInfo()
    st = lib().kkt_refactor_inertia(h, _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x), _dptr(sigma_s), float(gamma),
                                    C.byref(opts) if opts is not None else None, C.byref(ii), _stream(stream))
    if st not in (KKT_OK, 4):
        _err(st)
    return ii.as_dict()


def kkt_solve_augmented(h, r1, r2, r4, dx, ds, dz, max_iter: int = 10, tol: float = 1e-14, stream=None) -> dict:
    ro = RefineOpts(max_iter, tol)
    ai = AugInfo()
    st = lib().kkt_solve_augmented(h, _dptr(r1), _dptr(r2), _dptr(r4), _dptr(dx), _dptr(ds), _dptr(dz),
                                   C.byref(ro), C.byref(ai), _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return ai.as_dict()


def kkt_status_sync(h):
    fi = FactorInfo()
    st = lib().kkt_status_sync(h, C.byref(fi))
    return st, fi.bad_col


def kkt_solve(h, b, x, max_iter: int = 10, tol: float = 1e-14, info: bool = True, stream=None):
    ro = RefineOpts(max_iter, tol)
    si = SolveInfo()
    st = lib().kkt_solve(h, _dptr(b), _dptr(x), C.byref(ro), C.byref(si) if info else None, _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return si.as_dict() if info else None


def kkt_solve_noalloc(h, b, x, max_iter: int = 10, tol: float = 1e-14, info: bool = True, stream=None):
    ro = RefineOpts(max_iter, tol)
    si = SolveInfo()
    st = lib().kkt_solve_noalloc(h, _dptr(b), _dptr(x), C.byref(ro), C.byref(si) if info else None,
                                 _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return si.as_dict() if info else None


def kkt_cg_opts_default() -> CgOpts:
    o = CgOpts()
    lib().kkt_cg_opts_default(C.byref(o))
    return o


def kkt_cg_schur(h, f, g, dx, dy, tol: float = 1e-10, maxit: int = 200, eta_tol: float = 0.0, info: bool = True,
                 stream=None):
    o = CgOpts(float(tol), int(maxit), float(eta_tol))
    ci = CgInfo()
    st = lib().kkt_cg_schur(h, _dptr(f), _dptr(g), C.byref(o), _dptr(dx), _dptr(dy),
                            C.byref(ci) if info else None, _stream(stream))
    if st not in (KKT_OK, 6, 7):
        _err(st)
    return ci.as_dict() if info else None


def kkt_ipm_qp(h, w_vals, j_vals, c, u, x, s, z, tol: float = 1e-8, maxit: int = 100, sigma: float = 0.1,
               tau_min: float = 0.99, stream=None) -> dict:
    o = IpmOpts(float(tol), int(maxit), float(sigma), float(tau_min))
    ii = IpmInfo()
    st = lib().kkt_ipm_qp(h, _dptr(w_vals), _dptr(j_vals), _dptr(c), _dptr(u), _dptr(x), _dptr(s), _dptr(z),
                          C.byref(o), C.byref(ii), _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return ii.as_dict()


def kkt_factor_keep_augmented(h, enable: bool = True):
    _err(lib().kkt_factor_keep_augmented(h, 1 if enable else 0))


def kkt_factor_set_equality_rows(h, rows):
    r = _i32(rows if rows is not None else [])
    _err(lib().kkt_factor_set_equality_rows(h, _ptr_np(r) if len(r) else None, int(len(r))))


def kkt_matvec(h, x, y, stream=None):
    _err(lib().kkt_matvec(h, _dptr(x), _dptr(y), _stream(stream)))


def kkt_factor_set_timing(h, enable: bool):
    _err(lib().kkt_factor_set_timing(h, 1 if enable else 0))


def kkt_factor_read_timing(h) -> dict:
    t = Timing()
    _err(lib().kkt_factor_read_timing(h, C.byref(t)))
    return t.as_dict()


def kkt_factor_set_schedule(h, schedule: int):
    _err(lib().kkt_factor_set_schedule(h, int(schedule)))


def kkt_factor_set_update_split(h, max_fronts: int, min_rows: int):
    _err(lib().kkt_factor_set_update_split(h, int(max_fronts), int(min_rows)))


def kkt_factor_set_small_fronts(h, max_cols: int):
    _err(lib().kkt_factor_set_small_fronts(h, int(max_cols)))


# ---------------------------------------------------------------------------
# handle wrappers
# ---------------------------------------------------------------------------

class Symbolic:
    """Symbolic analysis of one (W, J) pattern (host only)."""

    def __init__(self, n, m, w_rowptr, w_colind, j_rowptr, j_colind, ordering=ORDER_AUTO, nd_leaf=0,
                 max_super=0, relax_small=0, relax_frac=-1.0, front_lds_max=0):
        opt = Options(ordering, nd_leaf, max_super, relax_small, relax_frac, front_lds_max)
        self.n, self.m = int(n), int(m)
        self.h = kkt_symbolic_analyze(self.n, self.m, w_rowptr, w_colind, j_rowptr, j_colind, opt)

    @classmethod
    def from_pattern(cls, pat, **kw):
        return cls(pat.n, pat.m, pat.w_rowptr, pat.w_colind, pat.j_rowptr, pat.j_colind, **kw)

    def stats(self) -> dict:
        return kkt_symbolic_get_stats(self.h)

    def perm(self) -> np.ndarray:
        return kkt_symbolic_get_perm(self.h, self.n)

    def supernodes(self):
        return kkt_symbolic_get_supernodes(self.h, self.stats()["nsuper"])

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            kkt_symbolic_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Factor:
    """Device factor of one pattern (keeps a reference to its Symbolic)."""

    def __init__(self, sym: Symbolic):
        self.sym = sym
        self.h = kkt_factor_create(sym.h)

    def refactor(self, w_vals, j_vals, sigma_x, sigma_s=None, gamma=0.0, stream=None):
        kkt_refactor(self.h, w_vals, j_vals, sigma_x, sigma_s, gamma, stream)

    def refactor_inertia(self, w_vals, j_vals, sigma_x, sigma_s=None, gamma=0.0, opts=None, stream=None):
        return kkt_refactor_inertia(self.h, w_vals, j_vals, sigma_x, sigma_s, gamma, opts, stream)

    def solve_augmented(self, r1, r2, r4, dx, ds, dz, max_iter=10, tol=1e-14, stream=None):
        return kkt_solve_augmented(self.h, r1, r2, r4, dx, ds, dz, max_iter, tol, stream)

    def status(self):
        return kkt_status_sync(self.h)

    def solve(self, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
        return kkt_solve(self.h, b, x, max_iter, tol, info, stream)

    def solve_noalloc(self, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
        return kkt_solve_noalloc(self.h, b, x, max_iter, tol, info, stream)

    def cg_schur(self, f, g, dx, dy, tol=1e-10, maxit=200, eta_tol=0.0, info=True, stream=None):
        return kkt_cg_schur(self.h, f, g, dx, dy, tol, maxit, eta_tol, info, stream)

    def ipm_qp(self, w_vals, j_vals, c, u, x, s, z, **kw):
        return kkt_ipm_qp(self.h, w_vals, j_vals, c, u, x, s, z, **kw)

    def keep_augmented(self, enable=True):
        kkt_factor_keep_augmented(self.h, enable)

    def set_equality_rows(self, rows):
        kkt_factor_set_equality_rows(self.h, rows)

    def matvec(self, x, y, stream=None):
        kkt_matvec(self.h, x, y, stream)

    def set_timing(self, enable=True):
        kkt_factor_set_timing(self.h, enable)

    def read_timing(self) -> dict:
        return kkt_factor_read_timing(self.h)

    def set_schedule(self, schedule: int):
        kkt_factor_set_schedule(self.h, schedule)

    def set_update_split(self, max_fronts: int, min_rows: int):
        kkt_factor_set_update_split(self.h, max_fronts, min_rows)

    def set_small_fronts(self, max_cols: int):
        kkt_factor_set_small_fronts(self.h, max_cols)

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            kkt_factor_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

def kkt_batch_create(sym_handles):
    arr = (C.c_void_p * len(sym_handles))(*[h.value for h in sym_handles])
    h = C.c_void_p()
    _err(lib().kkt_batch_create(len(sym_handles), arr, C.byref(h)))
    return h


def kkt_batch_offsets(h, count: int):
    outs = [np.empty(count + 1, dtype=np.int64) for _ in range(4)]
    _err(lib().kkt_batch_offsets(h, *[_ptr_np(o) for o in outs]))
    return dict(zip(("n", "m", "w", "j"), outs))


def kkt_batch_refactor(h, w_vals, j_vals, sigma_x, sigma_s, stream=None):
    _err(lib().kkt_batch_refactor(h, _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x), _dptr(sigma_s), _stream(stream)))


def kkt_batch_solve(h, count, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
    ro = RefineOpts(max_iter, tol)
    infos = (SolveInfo * count)()
    st = lib().kkt_batch_solve(h, _dptr(b), _dptr(x), C.byref(ro), infos if info else None, _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return [i.as_dict() for i in infos] if info else None


def kkt_batch_status(h, count):
    st = np.zeros(count, dtype=np.int32)
    bad = np.zeros(count, dtype=np.int32)
    lib().kkt_batch_status(h, _ptr_np(st), _ptr_np(bad))
    return st, bad


def kkt_batch_set_schedule(h, schedule: int):
    _err(lib().kkt_batch_set_schedule(h, int(schedule)))


def kkt_batch_capture(h, w_vals, j_vals, sigma_x, sigma_s, b, x, max_iter=10, tol=1e-14, rounds=2):
    ro = RefineOpts(max_iter, tol)
    _err(lib().kkt_batch_capture(h, _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x), _dptr(sigma_s), _dptr(b),
                                 _dptr(x), C.byref(ro), int(rounds)))


def kkt_batch_replay(h, count, info=True, stream=None):
    infos = (SolveInfo * count)()
    st = lib().kkt_batch_replay(h, infos if info else None, _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return [i.as_dict() for i in infos] if info else None


class Batch:
    """Batched refactor + solve of many instances (concatenated device arrays)."""

    def __init__(self, syms):
        self.syms = list(syms)
        self.count = len(self.syms)
        self.h = kkt_batch_create([s.h for s in self.syms])
        self.ofs = kkt_batch_offsets(self.h, self.count)

    def refactor(self, w_vals, j_vals, sigma_x, sigma_s, stream=None):
        kkt_batch_refactor(self.h, w_vals, j_vals, sigma_x, sigma_s, stream)

    def solve(self, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
        return kkt_batch_solve(self.h, self.count, b, x, max_iter, tol, info, stream)

    def status(self):
        return kkt_batch_status(self.h, self.count)

    def set_schedule(self, schedule: int):
        kkt_batch_set_schedule(self.h, schedule)

    def set_update_split(self, max_fronts: int, min_rows: int):
        _err(lib().kkt_batch_set_update_split(self.h, int(max_fronts), int(min_rows)))

    def set_small_fronts(self, max_cols: int):
        _err(lib().kkt_batch_set_small_fronts(self.h, int(max_cols)))

    def capture(self, w_vals, j_vals, sigma_x, sigma_s, b, x, max_iter=10, tol=1e-14, rounds=2):
        """Record refactor + solve as a graph bound to these arrays (kept alive here)."""
        kkt_batch_capture(self.h, w_vals, j_vals, sigma_x, sigma_s, b, x, max_iter, tol, rounds)
        self._graph_args = (w_vals, j_vals, sigma_x, sigma_s, b, x)

    def replay(self, info=True, stream=None):
        return kkt_batch_replay(self.h, self.count, info, stream)

    def set_timing(self, enable=True):
        _err(lib().kkt_batch_set_timing(self.h, 1 if enable else 0))

    def read_timing(self) -> dict:
        t = Timing()
        _err(lib().kkt_batch_read_timing(self.h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kkt_batch_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# stage-structured solver (block cyclic reduction)
# ---------------------------------------------------------------------------

def kkt_stagewise_create(sym_handles, stage_ptrs):
    count = len(sym_handles)
    sps = [np.ascontiguousarray(sp, dtype=np.int32) for sp in stage_ptrs]
    arr = (C.c_void_p * count)(*[h.value for h in sym_handles])
    ptrs = (C.c_void_p * count)(*[sp.ctypes.data for sp in sps])
    ns = np.array([len(sp) - 1 for sp in sps], dtype=np.int32)
    h = C.c_void_p()
    _err(lib().kkt_stagewise_create(count, arr, ptrs, _ptr_np(ns), C.byref(h)))
    return h


def kkt_stagewise_refactor(h, w_vals, j_vals, sigma_x, sigma_s, stream=None):
    _err(lib().kkt_stagewise_refactor(h, _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x), _dptr(sigma_s),
                                      _stream(stream)))


def kkt_stagewise_status(h, count):
    st = np.zeros(count, dtype=np.int32)
    bad = np.zeros(count, dtype=np.int32)
    lib().kkt_stagewise_status(h, _ptr_np(st), _ptr_np(bad))
    return st, bad


def kkt_stagewise_solve(h, count, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
    ro = RefineOpts(max_iter, tol)
    infos = (SolveInfo * count)()
    st = lib().kkt_stagewise_solve(h, _dptr(b), _dptr(x), C.byref(ro), infos if info else None, _stream(stream))
    if st not in (KKT_OK, 6):
        _err(st)
    return [i.as_dict() for i in infos] if info else None


class Stagewise:
    """Block-tridiagonal K of stage-structured patterns, factored by block cyclic reduction.

    ``stage_ptrs[q]`` holds the stage starts of instance q (0 .. n). Values and
    vectors are concatenated in instance order, as for :class:`Batch`.
    """

    def __init__(self, syms, stage_ptrs):
        self.syms = list(syms)
        self.count = len(self.syms)
        self.h = kkt_stagewise_create([s.h for s in self.syms], stage_ptrs)

    def refactor(self, w_vals, j_vals, sigma_x, sigma_s, stream=None):
        kkt_stagewise_refactor(self.h, w_vals, j_vals, sigma_x, sigma_s, stream)

    def solve(self, b, x, max_iter=10, tol=1e-14, info=True, stream=None):
        return kkt_stagewise_solve(self.h, self.count, b, x, max_iter, tol, info, stream)

    def status(self):
        return kkt_stagewise_status(self.h, self.count)

    def set_timing(self, enable=True):
        _err(lib().kkt_stagewise_set_timing(self.h, 1 if enable else 0))

    def read_timing(self) -> dict:
        t = Timing()
        _err(lib().kkt_stagewise_read_timing(self.h, C.byref(t)))
        return t.as_dict()

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kkt_stagewise_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# served form
# ---------------------------------------------------------------------------

class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_wave", C.c_int32), ("workers", C.c_int32),
                ("refine_max_iter", C.c_int32), ("refine_tol", C.c_double), ("linger_us", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64), ("waves", C.c_int64),
                ("mean_wave", C.c_double), ("p50_s", C.c_double), ("p99_s", C.c_double),
                ("mean_queue_s", C.c_double), ("mean_service_s", C.c_double), ("throughput", C.c_double),
                ("window_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """Request loop over resident patterns (continuous batching)."""

    def __init__(self, hbm_budget=8 << 30, max_wave=64, workers=2, refine_max_iter=10, refine_tol=1e-14,
                 linger_us=0.0):
        o = ServerOpts()
        lib().kkt_server_opts_default(C.byref(o))
        o.hbm_budget, o.max_wave, o.workers = int(hbm_budget), int(max_wave), int(workers)
        o.refine_max_iter, o.refine_tol, o.linger_us = int(refine_max_iter), float(refine_tol), float(linger_us)
        self.h = C.c_void_p()
        _err(lib().kkt_server_create(C.byref(o), C.byref(self.h)))
        self.keep = []

    def register(self, sym: Symbolic) -> int:
        pid = C.c_int32()
        _err(lib().kkt_server_register(self.h, sym.h, C.byref(pid)))
        self.keep.append(sym)
        return pid.value

    def submit(self, pid, w_vals, j_vals, sigma_x, sigma_s, b, x, stream=None) -> int:
        """Queues a request ordered after the work already enqueued on `stream` (default: torch's
        current stream), so inputs and x written there just before are seen complete."""
        t = C.c_int64()
        _err(lib().kkt_server_submit(self.h, int(pid), _dptr(w_vals), _dptr(j_vals), _dptr(sigma_x),
                                     _dptr(sigma_s), _dptr(b), _dptr(x), _stream(stream), C.byref(t)))
        return t.value

    def wait(self, ticket):
        si = SolveInfo()
        lat = C.c_double()
        st = lib().kkt_server_wait(self.h, int(ticket), C.byref(si), C.byref(lat))
        d = si.as_dict()
        d["status"] = st
        d["latency_s"] = lat.value
        return d

    def stats(self) -> dict:
        s = ServerStats()
        _err(lib().kkt_server_get_stats(self.h, C.byref(s)))
        return s.as_dict()

    def reset_stats(self):
        _err(lib().kkt_server_reset_stats(self.h))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().kkt_server_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
