"""Dense FP64 oracle: explicit KKT systems, Bunch-Kaufman LDL^T, evaluators.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references are to Pacaud & Shin, "GPU-accelerated dynamic nonlinear
optimization with ExaModels and MadNLP" (arXiv 2403.15913):
  * augmented KKT system, eq. (kkt:augmented), section "Augmented KKT system";
  * condensed system and condensed matrix K = W + delta_x + H^T D_s H,
    eq. (kkt:condensed), section "Condensed KKT system";
  * Lifted-KKT: every constraint treated as an inequality, K d_x = rhs,
    eq. (liftedkkt), section "Solution 1: Lifted-KKT";
  * HyKKT: K_gamma = K + gamma G^T G, the equivalent system eq. (hykkt) and
    the Schur-complement system eq. (schurcomp), section "Solution 2: HyKKT";
  * inertia condition eq. (inertia) and its condensed equivalent (the
    Haynsworth statement after eq. (kkt:condensed)).

Notation used here (the library's): J is the constraint Jacobian, Sigma_x the
primal diagonal (delta_x I plus bound terms), Sigma_s the slack diagonal
D_s = S^{-1} V, and gamma the augmented-Lagrangian weight.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

ALPHA_BK = (1.0 + np.sqrt(17.0)) / 8.0


# --------------------------------------------------------------------------
# Explicit matrices
# --------------------------------------------------------------------------

def w_full(pat, vals) -> sp.csr_matrix:
    """Symmetric W from its lower-triangle CSR."""
    L = sp.csr_matrix((vals.w_vals, pat.w_colind, pat.w_rowptr), shape=(pat.n, pat.n))
    return (L + L.T - sp.diags(L.diagonal())).tocsr()


def jacobian(pat, vals) -> sp.csr_matrix:
    return sp.csr_matrix((vals.j_vals, pat.j_colind, pat.j_rowptr), shape=(pat.m, pat.n))


def condensed(pat, vals, row_weight) -> sp.csr_matrix:
    """K = W + diag(Sigma_x) + J^T diag(d) J.

    d = Sigma_s gives the Lifted-KKT condensed matrix (eq. (kkt:condensed)
    with every constraint an inequality, eq. (liftedkkt)); d = gamma * ones
    gives K_gamma of eq. (hykkt) with no inequality rows.
    """
    J = jacobian(pat, vals)
    d = np.broadcast_to(np.asarray(row_weight, dtype=np.float64), (pat.m,))
    return (w_full(pat, vals) + sp.diags(vals.sigma_x) + J.T @ sp.diags(d) @ J).tocsr()


def lifted_saddle(pat, vals) -> np.ndarray:
    """2x2 quasi-definite form [[W+Sx, J^T], [J, -Ss^{-1}]] (slack block eliminated).

    With right-hand side [b; 0] its x-part is the Lifted-KKT solution: the
    second row gives y = Ss J x and substituting it back yields K x = b.
    """
    W = w_full(pat, vals).toarray() + np.diag(vals.sigma_x)
    J = jacobian(pat, vals).toarray()
    return np.block([[W, J.T], [J, -np.diag(1.0 / vals.sigma_s)]])


def lifted_augmented(pat, vals) -> np.ndarray:
    """Augmented system of eq. (kkt:augmented) with no equality rows (m_e = 0).

    Unknowns (d_x, d_s, d_z); blocks [[W+Sx, 0, H^T], [0, D_s, I], [H, I, 0]]
    with H = J and D_s = Sigma_s.
    """
    n, m = pat.n, pat.m
    W = w_full(pat, vals).toarray() + np.diag(vals.sigma_x)
    H = jacobian(pat, vals).toarray()
    Z = np.zeros
    return np.block([[W, Z((n, m)), H.T],
                     [Z((m, n)), np.diag(vals.sigma_s), np.eye(m)],
                     [H, np.eye(m), Z((m, m))]])


def condensed_rhs(pat, vals, r1, r2, r4) -> np.ndarray:
    """Right-hand side of the condensed solve, -(r1 + H^T (D_s r4 - r2)) (eq. (kkt:condensed))."""
    J = jacobian(pat, vals)
    return -(r1 + J.T @ (vals.sigma_s * r4 - r2))


def recover_slack_steps(pat, vals, dx, r2, r4):
    """d_s = -r4 - H d_x and d_z = -r2 - D_s d_s (stated after eq. (kkt:condensed))."""
    J = jacobian(pat, vals)
    ds = -r4 - J @ dx
    dz = -r2 - vals.sigma_s * ds
    return ds, dz


def lifted_augmented_regularized(pat, vals, delta: float) -> np.ndarray:
    """The augmented system of eq. (kkt:augmented) (no equality rows) with the
    primal regularisation delta added to the Hessian block only, the form whose
    condensation is the condensed matrix K = W + delta_x I + H^T D_s H as the
    paper writes it after eq. (kkt:condensed)."""
    A = lifted_augmented(pat, vals)
    A[:pat.n, :pat.n] += delta * np.eye(pat.n)
    return A


# Inertia correction: the regularisation (delta_x) is raised until the
# augmented system has the inertia of eq. (inertia), (n + m, 0, m) with no
# equality rows. The paper fixes no update rule; this is the rule of the
# filter line-search interior-point method (Waechter & Biegler 2006, its
# inertia-correction algorithm): try delta = 0; on failure start from
# delta_first (no earlier success) or from max(delta_min, kappa_minus *
# delta_last); multiply by kappa_plus_first (no earlier success) or
# kappa_plus until the inertia is right or delta exceeds delta_max.
INERTIA_DEFAULTS = dict(delta_first=1e-4, delta_min=1e-20, delta_max=1e40, kappa_minus=1.0 / 3.0,
                        kappa_plus=8.0, kappa_plus_first=100.0)


def augmented_inertia_ok(pat, vals, delta: float) -> bool:
    """Inertia of the regularised augmented system by Bunch-Kaufman equals (n + m, 0, m)."""
    return bunch_kaufman(lifted_augmented_regularized(pat, vals, delta)).inertia() == (pat.n + pat.m, 0, pat.m)


def inertia_correction(pat, vals, delta_last: float = 0.0, **opts):
    """Returns (delta, trials, delta_last_after); delta is None when delta_max is exceeded."""
    o = dict(INERTIA_DEFAULTS, **opts)
    trials = [0.0]
    if augmented_inertia_ok(pat, vals, 0.0):
        return 0.0, trials, delta_last
    delta = o["delta_first"] if delta_last == 0.0 else max(o["delta_min"], o["kappa_minus"] * delta_last)
    while delta <= o["delta_max"]:
        trials.append(delta)
        if augmented_inertia_ok(pat, vals, delta):
            return delta, trials, delta
        delta *= o["kappa_plus_first"] if delta_last == 0.0 else o["kappa_plus"]
    return None, trials, delta_last


def hykkt_saddle(pat, vals, gamma: float = 0.0) -> np.ndarray:
    """[[K0 + gamma J^T J, J^T], [J, 0]] with K0 = W + Sigma_x (eq. (hykkt); gamma=0 is eq. (kkt:condensed))."""
    K0 = w_full(pat, vals).toarray() + np.diag(vals.sigma_x)
    J = jacobian(pat, vals).toarray()
    return np.block([[K0 + gamma * (J.T @ J), J.T], [J, np.zeros((pat.m, pat.m))]])


def split_rows(pat, vals, eq_rows):
    """(G, H, D_s): the equality rows of J (in the order given), the remaining
    (inequality) rows in ascending order, and their slack weights."""
    J = jacobian(pat, vals)
    eq = np.asarray(eq_rows, dtype=np.int64)
    mask = np.zeros(pat.m, dtype=bool)
    mask[eq] = True
    ineq = np.nonzero(~mask)[0]
    return J[eq].toarray(), J[ineq].toarray(), vals.sigma_s[ineq], eq, ineq


def general_hykkt_saddle(pat, vals, eq_rows, gamma: float = 0.0) -> np.ndarray:
    """[[K_k + gamma G^T G, G^T], [G, 0]] of eq. (hykkt) with the condensed
    matrix K_k = W + Sigma_x + H^T D_s H of eq. (kkt:condensed): G the equality
    rows of J, H the inequality rows with D_s their Sigma_s."""
    G, H, ds, _, _ = split_rows(pat, vals, eq_rows)
    Kk = w_full(pat, vals).toarray() + np.diag(vals.sigma_x) + H.T @ (ds[:, None] * H)
    return np.block([[Kk + gamma * (G.T @ G), G.T], [G, np.zeros((len(G), len(G)))]])


def general_augmented(pat, vals, eq_rows) -> np.ndarray:
    """The augmented system of eq. (kkt:augmented) with equality rows G and
    inequality rows H: unknowns (d_x, d_s, d_y, d_z)."""
    G, H, ds, _, _ = split_rows(pat, vals, eq_rows)
    n, me, mi = pat.n, len(G), len(H)
    W = w_full(pat, vals).toarray() + np.diag(vals.sigma_x)
    Z = np.zeros
    return np.block([[W, Z((n, mi)), G.T, H.T],
                     [Z((mi, n)), np.diag(ds), Z((mi, me)), np.eye(mi)],
                     [G, Z((me, mi)), Z((me, me)), Z((me, mi))],
                     [H, np.eye(mi), Z((mi, me)), Z((mi, mi))]])


def hykkt_rhs(pat, vals, f, g, gamma: float) -> np.ndarray:
    """[f + gamma J^T g; g]: the r_gamma shift of eq. (hykkt) in the positive-sign convention."""
    J = jacobian(pat, vals)
    return np.concatenate([f + gamma * (J.T @ g), g])


# --------------------------------------------------------------------------
# Bunch-Kaufman LDL^T (symmetric indefinite, 1x1 / 2x2 pivots)
# --------------------------------------------------------------------------

class BKFactor:
    """P A P^T = L D L^T with L unit lower triangular, D block diagonal."""

    def __init__(self, perm, L, blocks):
        self.perm = perm      # P A P^T = A[perm][:, perm]
        self.L = L
        self.blocks = blocks  # list of (start, size, block)

    def solve(self, b: np.ndarray) -> np.ndarray:
        y = _unit_lower_solve(self.L, b[self.perm])
        z = np.empty_like(y)
        for k, s, blk in self.blocks:
            if s == 1:
                z[k] = y[k] / blk[0, 0]
            else:
                z[k:k + 2] = np.linalg.solve(blk, y[k:k + 2])
        w = _unit_upper_solve(self.L.T, z)
        x = np.empty_like(w)
        x[self.perm] = w
        return x

    def inertia(self):
        """(n_plus, n_zero, n_minus) from the D blocks (Sylvester's law of inertia)."""
        pos = zero = neg = 0
        for _, s, blk in self.blocks:
            ev = [blk[0, 0]] if s == 1 else np.linalg.eigvalsh(blk)
            for e in ev:
                if e > 0:
                    pos += 1
                elif e < 0:
                    neg += 1
                else:
                    zero += 1
        return pos, zero, neg


def _unit_lower_solve(L, b):
    x = b.astype(np.float64).copy()
    for i in range(len(x)):
        x[i] -= L[i, :i] @ x[:i]
    return x


def _unit_upper_solve(U, b):
    x = b.astype(np.float64).copy()
    n = len(x)
    for i in range(n - 1, -1, -1):
        x[i] -= U[i, i + 1:] @ x[i + 1:]
    return x


def bunch_kaufman(A: np.ndarray) -> BKFactor:
    """Bunch-Kaufman diagonal pivoting (Bunch & Kaufman 1977; Golub & Van Loan sec. 4.4).

    At step k, with lam the largest |A[i,k]| below the diagonal (row r):
      |A[k,k]| >= alpha lam                     -> 1x1 pivot, no interchange;
      else sig = largest off-diagonal |A[i,r]|, i >= k:
        |A[k,k]| sig >= alpha lam^2             -> 1x1 pivot, no interchange;
        |A[r,r]| >= alpha sig                    -> 1x1 pivot after swapping k and r;
        otherwise                                -> 2x2 pivot after swapping k+1 and r,
    with alpha = (1 + sqrt(17)) / 8. A zero pivot column is recorded as a 1x1
    zero block (the matrix is then singular and the inertia has n_zero > 0).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    perm = np.arange(n)
    L = np.eye(n)
    blocks = []

    def swap(i, j, k):
        # symmetric interchange of rows/columns i and j (both >= k); only the
        # already computed columns 0..k-1 of L move with the rows
        if i == j:
            return
        A[[i, j], :] = A[[j, i], :]
        A[:, [i, j]] = A[:, [j, i]]
        perm[[i, j]] = perm[[j, i]]
        L[[i, j], :k] = L[[j, i], :k]

    k = 0
    while k < n:
        akk = abs(A[k, k])
        size = 1
        if k < n - 1:
            col = np.abs(A[k + 1:, k])
            r = int(np.argmax(col)) + k + 1
            lam = col[r - k - 1]
            if max(akk, lam) == 0.0:
                size = 1
            elif akk >= ALPHA_BK * lam:
                size = 1
            else:
                others = np.abs(A[k:, r])
                others[r - k] = 0.0
                sig = others.max()
                if akk * sig >= ALPHA_BK * lam * lam:
                    size = 1
                elif abs(A[r, r]) >= ALPHA_BK * sig:
                    swap(k, r, k)
                    size = 1
                else:
                    swap(k + 1, r, k)
                    size = 2
        if size == 1:
            d = A[k, k]
            blocks.append((k, 1, np.array([[d]])))
            if d != 0.0 and k < n - 1:
                l = A[k + 1:, k] / d
                A[k + 1:, k + 1:] -= np.outer(l, A[k + 1:, k])
                L[k + 1:, k] = l
            k += 1
        else:
            E = A[k:k + 2, k:k + 2].copy()
            blocks.append((k, 2, E))
            if k + 2 < n:
                C = A[k + 2:, k:k + 2]
                CEinv = np.linalg.solve(E, C.T).T   # E symmetric
                A[k + 2:, k + 2:] -= CEinv @ C.T
                L[k + 2:, k:k + 2] = CEinv
            k += 2
    return BKFactor(perm, L, blocks)


# --------------------------------------------------------------------------
# Reference solutions
# --------------------------------------------------------------------------

def lifted_solution(pat, vals, b):
    """x* of K x = b via Bunch-Kaufman on the 2x2 quasi-definite form; also its inertia."""
    F = bunch_kaufman(lifted_saddle(pat, vals))
    sol = F.solve(np.concatenate([b, np.zeros(pat.m)]))
    return sol[:pat.n], F.inertia()


def hykkt_solution(pat, vals, f, g, gamma: float = 0.0):
    """(dx*, dy*) of [[K0 + gamma J^T J, J^T], [J, 0]] [dx; dy] = [f + gamma J^T g; g]; also the inertia."""
    F = bunch_kaufman(hykkt_saddle(pat, vals, gamma))
    sol = F.solve(hykkt_rhs(pat, vals, f, g, gamma))
    return sol[:pat.n], sol[pat.n:], F.inertia()


# --------------------------------------------------------------------------
# Residual evaluators
# --------------------------------------------------------------------------

def _inf_norm_matrix(A) -> float:
    if sp.issparse(A):
        return float(np.abs(A).sum(axis=1).max()) if A.shape[0] else 0.0
    return float(np.abs(A).sum(axis=1).max()) if A.shape[0] else 0.0


def backward_errors(A, x, b) -> dict:
    """Normwise (Rigal-Gaches) and componentwise (Oettli-Prager) backward errors.

    eta   = ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf)
    omega = max_i |b - A x|_i / (|A| |x| + |b|)_i   (0/0 taken as 0)
    relres = ||b - A x||_inf / ||b||_inf
    """
    r = b - A @ x
    absA = abs(A)
    denom_c = absA @ np.abs(x) + np.abs(b)
    rabs = np.abs(r)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(denom_c > 0, rabs / np.where(denom_c > 0, denom_c, 1.0), np.where(rabs > 0, np.inf, 0.0))
    nb = np.abs(b).max() if len(b) else 0.0
    denom = _inf_norm_matrix(A) * (np.abs(x).max() if len(x) else 0.0) + nb
    return dict(eta=float(rabs.max() / denom) if denom > 0 else 0.0,
                omega=float(q.max()) if len(q) else 0.0,
                relres=float(rabs.max() / nb) if nb > 0 else float(rabs.max()))


def forward_error(x, xstar) -> float:
    """Normwise relative forward error ||x - x*||_inf / ||x*||_inf."""
    return float(np.linalg.norm(x - xstar, np.inf) / np.linalg.norm(xstar, np.inf))


def componentwise_error(x, xstar, floor: float = 1e-12) -> float:
    """max_i |x_i - x*_i| / (|x*_i| + floor ||x*||_inf).

    The relative error of every entry, with entries far below the largest
    one measured against floor * ||x*||_inf instead of themselves; a value
    <= tol means |x - x*| <= tol |x*| + tol * floor ||x*||_inf entrywise.
    """
    x = np.asarray(x, dtype=np.float64)
    xstar = np.asarray(xstar, dtype=np.float64)
    if len(xstar) == 0:
        return 0.0
    den = np.abs(xstar) + floor * np.abs(xstar).max()
    d = np.abs(x - xstar)
    with np.errstate(divide="ignore", invalid="ignore"):
        q = np.where(den > 0, d / np.where(den > 0, den, 1.0), np.where(d > 0, np.inf, 0.0))
    return float(q.max())


def hykkt_backward_errors(pat, vals, dx, dy, f, g) -> dict:
    """Backward errors of (dx, dy) on [[K0, J^T], [J, 0]] [dx; dy] = [f; g]."""
    J = jacobian(pat, vals)
    K0 = (w_full(pat, vals) + sp.diags(vals.sigma_x)).tocsr()
    A = sp.bmat([[K0, J.T], [J, None]], format="csr")
    return backward_errors(A, np.concatenate([dx, dy]), np.concatenate([f, g]))


# --------------------------------------------------------------------------
# Schur complement of the HyKKT system
# --------------------------------------------------------------------------

def schur_dense(pat, vals, gamma: float) -> np.ndarray:
    """S_gamma = J K_gamma^{-1} J^T (eq. (schurcomp)), formed densely."""
    Kg = condensed(pat, vals, gamma).toarray()
    J = jacobian(pat, vals).toarray()
    return J @ np.linalg.solve(Kg, J.T)


def schur_eigs_closed_form(eig_s0: np.ndarray, gamma: float) -> np.ndarray:
    """Eigenvalues of S_gamma from those of S_0 = J K0^{-1} J^T.

    With K0 SPD and J of full row rank, the Sherman-Morrison-Woodbury
    identity gives S_gamma = (S_0^{-1} + gamma I)^{-1}, so each eigenvalue
    maps as lambda -> 1 / (gamma + 1/lambda); they tend to 1/gamma as gamma
    grows, which is the convergence statement after eq. (schurcomp).
    """
    return 1.0 / (gamma + 1.0 / eig_s0)


def cg_iteration_bound(kappa: float, tol: float) -> int:
    """Classical CG bound: iterations <= ceil(0.5 sqrt(kappa) ln(2/tol))."""
    return int(np.ceil(0.5 * np.sqrt(kappa) * np.log(2.0 / tol)))
