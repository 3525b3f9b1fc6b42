"""Parity gates shared by the GPU tests (the oracle's evaluators, fixed tolerances).

* ``assert_well_conditioned``: Sigma in [1e-2, 1e2]. Relative forward error
  ||x - x*||_inf / ||x*||_inf <= 1e-8, and entry by entry
  |x_i - x*_i| <= 1e-8 |x*_i| + 1e-12 ||x*||_inf.
* ``assert_cond_bounded``: wider Sigma ranges. Both x and x* are backward
  stable (eta ~ 1e-17), so their difference is bounded by the conditioning:
  ||x - x*|| / ||x*|| <= 1e-13 cond_2(K) (about 500 unit roundoffs times the
  condition number), with cond_2(K) = lambda_max / lambda_min of the SPD K
  computed by Lanczos iterations.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as sla

from oracle import dense as D

FE_WELL = 1e-8
CW_FLOOR = 1e-4          # 1e-8 * 1e-4 = 1e-12 of ||x*||_inf
COND_FACTOR = 1e-13


def assert_well_conditioned(x, xs, what=""):
    fe = D.forward_error(x, xs)
    cw = D.componentwise_error(x, xs, CW_FLOOR)
    assert fe <= FE_WELL and cw <= FE_WELL, (what, fe, cw)


def cond_spd(K) -> float:
    """cond_2 of a symmetric positive definite sparse matrix (extreme eigenvalues)."""
    K = K.tocsc()
    n = K.shape[0]
    if n <= 600:
        ev = np.linalg.eigvalsh(K.toarray())
        return float(ev[-1] / ev[0])
    hi = sla.eigsh(K, k=1, which="LA", return_eigenvectors=False, tol=1e-6)[0]
    lo = sla.eigsh(K, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-6)[0]
    return float(hi / lo)


def assert_cond_bounded(x, xs, K, what=""):
    fe = D.forward_error(x, xs)
    bound = COND_FACTOR * cond_spd(K)
    assert fe <= bound, (what, fe, bound)
