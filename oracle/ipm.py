"""Primal-dual interior-point method on a convex QP: TEST INFRASTRUCTURE ONLY.

Follows the paper's method (Pacaud & Shin, arXiv 2403.15913): section
"INTERIOR-POINT METHOD" (the smoothed KKT system eq. (smoothkkt) solved by
Newton's method, eq. (newtonstep), with a fraction-to-boundary step) and its
Newton step through the augmented system of eq. (kkt:augmented), condensed as
in eq. (kkt:condensed) and solved as Lifted-KKT (every constraint an
inequality, eq. (liftedkkt)).

Problem (a synthetic linear-quadratic MPC with analytic derivatives):
    min 1/2 x^T W x + c^T x   s.t.  J x <= u,
with slacks s: h(x) + s = 0, h(x) = J x - u, s >= 0, multipliers z (of the
equalities) and, the slack block eliminated, D_s = S^{-1} Z. One iteration:
    r1 = W x + c + J^T z,  r4 = J x + s - u,  gap = s^T z / m;
    stop when max(||r1||_inf / (1 + ||c||_inf), ||r4||_inf / (1 + ||u||_inf), gap) <= tol;
    mu = sigma * gap;  r2 = z - mu / s;
    the augmented system [[W, 0, J^T], [0, D_s, I], [J, I, 0]] d = -[r1; r2; r4]
    condensed: K dx = -(r1 + J^T (D_s r4 - r2)), K = W + J^T D_s J;
    ds = -r4 - J dx, dz = -r2 - D_s ds;
    tau = max(tau_min, 1 - mu); the largest alpha_p <= 1 with s + alpha_p ds >= (1 - tau) s,
    and alpha_d <= 1 with z + alpha_d dz >= (1 - tau) z (fraction to the boundary);
    x += alpha_p dx, s += alpha_p ds, z += alpha_d dz.
The paper's interior-point solver also has a filter line search; on a convex
QP this method takes the fraction-to-boundary steps only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import dense
from . import sparse as S


def fraction_to_boundary(v: np.ndarray, dv: np.ndarray, tau: float) -> float:
    """Largest alpha in (0, 1] with v + alpha dv >= (1 - tau) v (v > 0)."""
    neg = dv < 0
    if not neg.any():
        return 1.0
    return float(min(1.0, (-tau * v[neg] / dv[neg]).min()))


def qp_ipm(W, c, J, u, x0, s0, z0, tol: float = 1e-8, maxit: int = 100, sigma: float = 0.1,
           tau_min: float = 0.99, record=None):
    """Returns (x, s, z, info); info: iterations, status ('ok' | 'maxit'), residuals."""
    W = sp.csr_matrix(W)
    J = sp.csr_matrix(J)
    m = J.shape[0]
    x, s, z = (np.array(a, dtype=np.float64) for a in (x0, s0, z0))
    cn, un = 1.0 + np.abs(c).max(), 1.0 + np.abs(u).max()
    status = "maxit"
    it = 0
    for it in range(maxit + 1):
        r1 = W @ x + c + J.T @ z
        r4 = J @ x + s - u
        gap = float(s @ z) / m
        err = max(np.abs(r1).max() / cn, np.abs(r4).max() / un, gap)
        if record is not None:
            record.append(dict(x=x.copy(), s=s.copy(), z=z.copy(), err=err))
        if err <= tol:
            status = "ok"
            break
        if it == maxit:
            break
        mu = sigma * gap
        r2 = z - mu / s
        ds_w = z / s
        K = (W + J.T @ sp.diags(ds_w) @ J).tocsr()
        rhs = -(r1 + J.T @ (ds_w * r4 - r2))
        M = S.SymCSR(K)
        F = S.LDL(M)
        if not F.ok or not (F.d() > 0).all():
            status = "not_spd"
            break
        dx, _ = S.refine(M, F, rhs)
        ds = -r4 - J @ dx
        dz = -r2 - ds_w * ds
        tau = max(tau_min, 1.0 - mu)
        ap = fraction_to_boundary(s, ds, tau)
        ad = fraction_to_boundary(z, dz, tau)
        x = x + ap * dx
        s = s + ap * ds
        z = z + ad * dz
    r1 = W @ x + c + J.T @ z
    r4 = J @ x + s - u
    return x, s, z, dict(iterations=it, status=status, r1=float(np.abs(r1).max()), r4=float(np.abs(r4).max()),
                         gap=float(s @ z) / m)


def qp_from_pattern(pat, vals, c, u):
    """(W, c, J, u) of the QP on a KKT pattern: W from its lower triangle, J its Jacobian."""
    return dense.w_full(pat, vals), c, dense.jacobian(pat, vals), u
