"""Sparse FP64 oracle front end (ctypes over ``sparse_ldl.c``): TEST INFRASTRUCTURE ONLY.

  * ``lifted_solve``       -- condensed sparse Cholesky (as L D L^T, all D > 0)
                              of K = W + Sigma_x + J^T Sigma_s J in the original
                              (stage-major) order, then Richardson refinement.
  * ``saddle_order``       -- symmetric ordering of a 2x2 saddle-point system that
                              places every constraint right after its last primal
                              variable, so that static pivots exist.
  * ``hykkt_saddle_solve`` -- sparse LDL^T of [[W+Sigma_x, J^T], [J, 0]] under that
                              ordering: the saddle-point solution and its inertia.
  * ``lifted_saddle_solve``-- the same on [[W+Sigma_x, J^T], [J, -Sigma_s^{-1}]].
  * ``hykkt_cg_solve``     -- Cholesky of K_gamma plus plain conjugate gradient on the
                              Schur complement (eq. (schurcomp)); used for timing and
                              for the CG iteration counts, never as the reference
                              solution of the saddle-point system.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import scipy.sparse as sp

from . import dense
from .build import LIB, build_oracle

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        L = C.CDLL(LIB)
        P, I64, I32, D = C.c_void_p, C.c_int64, C.c_int, C.c_double
        ptr = np.ctypeslib.ndpointer
        L.ora_ldl_factor.argtypes = [I32, P, P, P, P, C.POINTER(C.c_void_p), C.POINTER(C.c_int)]
        L.ora_ldl_factor.restype = I32
        L.ora_ldl_free.argtypes = [P]
        L.ora_ldl_nnz.argtypes = [P]
        L.ora_ldl_nnz.restype = I64
        L.ora_ldl_inertia.argtypes = [P, I32, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.ora_ldl_get_d.argtypes = [P, P]
        L.ora_ldl_get_parent.argtypes = [P, P]
        L.ora_ldl_get_colcounts.argtypes = [P, P]
        L.ora_ldl_solve.argtypes = [P, P, P, P]
        L.ora_refine.argtypes = [I32, P, P, P, P, P, P, I32, D, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.ora_refine.restype = I32
        L.ora_hykkt_cg.argtypes = [I32, I32, P, P, P, P, D, P, P, D, I32, P, P,
                                   C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.ora_hykkt_cg.restype = I32
        del ptr
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


class SymCSR:
    """Symmetric matrix kept as full CSR (both triangles), int64 row pointers."""

    def __init__(self, A):
        A = sp.csr_matrix(A)
        A.sum_duplicates()
        A.sort_indices()
        self.n = A.shape[0]
        self.indptr = np.ascontiguousarray(A.indptr, dtype=np.int64)
        self.indices = np.ascontiguousarray(A.indices, dtype=np.int32)
        self.data = np.ascontiguousarray(A.data, dtype=np.float64)
        self.A = A


class LDL:
    """Sparse L D L^T with static pivots under the symmetric ordering ``perm``."""

    def __init__(self, A, perm=None):
        self.M = A if isinstance(A, SymCSR) else SymCSR(A)
        n = self.M.n
        self.perm = np.ascontiguousarray(np.arange(n) if perm is None else perm, dtype=np.int32)
        h = C.c_void_p()
        bad = C.c_int(-1)
        self.status = lib().ora_ldl_factor(n, _p(self.M.indptr), _p(self.M.indices), _p(self.M.data),
                                           _p(self.perm), C.byref(h), C.byref(bad))
        self.h = h
        self.bad = bad.value
        self.ok = self.status == 0

    def __del__(self):
        if getattr(self, "h", None) and self.h.value and _lib is not None:
            _lib.ora_ldl_free(self.h)
            self.h = C.c_void_p()

    def solve(self, b):
        assert self.ok
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.empty_like(b)
        w = np.empty_like(b)
        lib().ora_ldl_solve(self.h, _p(b), _p(x), _p(w))
        return x

    def inertia(self, upto: int = -1):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        lib().ora_ldl_inertia(self.h, upto, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def d(self):
        out = np.empty(self.M.n)
        lib().ora_ldl_get_d(self.h, _p(out))
        return out

    def parent(self):
        out = np.empty(self.M.n, dtype=np.int32)
        lib().ora_ldl_get_parent(self.h, _p(out))
        return out

    def colcounts(self):
        """Strictly-lower entries per column of L (valid after a successful factor)."""
        out = np.empty(self.M.n, dtype=np.int32)
        lib().ora_ldl_get_colcounts(self.h, _p(out))
        return out

    def nnz(self) -> int:
        return int(lib().ora_ldl_nnz(self.h))


def refine(M: SymCSR, F: LDL, b, maxit: int = 10, tol: float = 1e-14):
    """Richardson refinement with the stop rule omega <= tol, maxit, or omega not halving."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    x = np.empty_like(b)
    eta, om = C.c_double(), C.c_double()
    it = lib().ora_refine(M.n, _p(M.indptr), _p(M.indices), _p(M.data), F.h, _p(b), _p(x),
                          maxit, tol, C.byref(eta), C.byref(om))
    return x, dict(iters=it, eta=eta.value, omega=om.value)


def lifted_solve(pat, vals, b, maxit: int = 10, tol: float = 1e-14):
    """Lifted-KKT: condensed Cholesky of K = W + Sx + J^T Ss J plus refinement.

    Returns (x, info); info['spd'] is False (and x None) when a pivot is
    not positive, with info['bad_col'] the original index of that pivot.
    """
    M = SymCSR(dense.condensed(pat, vals, vals.sigma_s))
    F = LDL(M)
    if not F.ok:
        return None, dict(spd=False, bad_col=F.bad, status=F.status)
    d = F.d()
    if not (d > 0).all():
        k = int(np.argmax(~(d > 0)))
        return None, dict(spd=False, bad_col=int(F.perm[k]), status=1)
    x, info = refine(M, F, b, maxit, tol)
    info.update(spd=True, bad_col=-1, nnz_l=F.nnz())
    return x, info


def saddle_order(pat) -> np.ndarray:
    """Primal variables in their natural order; constraint i placed right after
    the largest column index of its row (constraints with an empty row last)."""
    n, m = pat.n, pat.m
    last = np.full(m, n, dtype=np.int64)
    rp = pat.j_rowptr
    nz = rp[1:] > rp[:-1]
    last[nz] = pat.j_colind[rp[1:][nz] - 1]
    # sort key: primal j -> (j, 0); constraint i -> (last_i, 1, i)
    keys_p = np.stack([np.arange(n), np.zeros(n, np.int64), np.zeros(n, np.int64)], 1)
    keys_c = np.stack([last, np.ones(m, np.int64), np.arange(m)], 1)
    keys = np.concatenate([keys_p, keys_c])
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    return order.astype(np.int32)


def _saddle(pat, vals, lower_right):
    J = dense.jacobian(pat, vals)
    K0 = (dense.w_full(pat, vals) + sp.diags(vals.sigma_x)).tocsr()
    return sp.bmat([[K0, J.T], [J, lower_right]], format="csr")


def hykkt_saddle_solve(pat, vals, f, g):
    """Sparse LDL^T of [[W+Sx, J^T], [J, 0]]: returns (dx, dy, inertia, ok)."""
    A = _saddle(pat, vals, sp.csr_matrix((pat.m, pat.m)))
    F = LDL(A, saddle_order(pat))
    if not F.ok:
        return None, None, F.inertia(), False
    sol = F.solve(np.concatenate([f, g]))
    return sol[:pat.n], sol[pat.n:], F.inertia(), True


def lifted_saddle_solve(pat, vals, b):
    """Sparse LDL^T of [[W+Sx, J^T], [J, -Ss^{-1}]] with rhs [b; 0]: returns (x, inertia, ok)."""
    A = _saddle(pat, vals, sp.diags(-1.0 / vals.sigma_s))
    F = LDL(A, saddle_order(pat))
    if not F.ok:
        return None, F.inertia(), False
    sol = F.solve(np.concatenate([b, np.zeros(pat.m)]))
    return sol[:pat.n], F.inertia(), True


def hykkt_cg_solve(pat, vals, f, g, gamma: float, tol: float = 1e-10, maxit: int = 200):
    """Cholesky of K_gamma = W + Sx + gamma J^T J, then CG on S_gamma = J K_gamma^{-1} J^T.

    Returns (dx, dy, info) with info = {status: 'ok'|'maxit'|'breakdown'|'not_spd',
    iters, true_res}.
    """
    Kg = SymCSR(dense.condensed(pat, vals, gamma))
    F = LDL(Kg)
    if not F.ok or not (F.d() > 0).all():
        return None, None, dict(status="not_spd", iters=0, true_res=np.inf)
    Jp = np.ascontiguousarray(pat.j_rowptr, dtype=np.int64)
    Ji = np.ascontiguousarray(pat.j_colind, dtype=np.int32)
    Jx = np.ascontiguousarray(vals.j_vals, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    dx = np.empty(pat.n)
    dy = np.empty(pat.m)
    it = C.c_int()
    res = C.c_double()
    st = lib().ora_hykkt_cg(pat.n, pat.m, _p(Jp), _p(Ji), _p(Jx), F.h, gamma, _p(f), _p(g),
                            tol, maxit, _p(dx), _p(dy), C.byref(it), C.byref(res))
    return dx, dy, dict(status={0: "ok", 6: "maxit", 7: "breakdown"}[st], iters=it.value, true_res=res.value)
