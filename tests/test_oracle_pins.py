"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

  * exact rational arithmetic (fractions) on tiny instances whose inputs are
    binary fractions, so float64 holds them exactly;
  * library brute force (numpy.linalg.solve / cholesky / eigvalsh);
  * the paper's identities: condensation (eq. (kkt:condensed)), the
    gamma-independence of the HyKKT system (eq. (hykkt)), the Haynsworth
    inertia equivalence stated after eq. (kkt:condensed), and the Schur
    spectrum tending to 1/gamma (after eq. (schurcomp));
  * special cases that reduce to textbook routines (Thomas algorithm,
    dense Cholesky, the range-space method at gamma = 0);
  * mistakes planted in the oracle must make at least one pin fail.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp

import kktgen
from oracle import dense as D
from oracle import sparse as S
from oracle import symbolic as Y

HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# exact helpers (independent of the oracle's algorithms)
# --------------------------------------------------------------------------

def frac_matrix(A):
    return [[Fraction(float(v)) for v in row] for row in np.asarray(A)]


def exact_solve(A, b):
    """Gauss-Jordan elimination over the rationals (any nonzero pivot)."""
    n = len(A)
    M = [row[:] + [Fraction(float(bi))] for row, bi in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def exact_det(A):
    """Bareiss fraction-free determinant (with row swaps)."""
    M = [row[:] for row in A]
    n = len(M)
    sign, prev = 1, Fraction(1)
    for k in range(n - 1):
        if M[k][k] == 0:
            p = next((r for r in range(k + 1, n) if M[r][k] != 0), None)
            if p is None:
                return Fraction(0)
            M[k], M[p] = M[p], M[k]
            sign = -sign
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                M[i][j] = (M[i][j] * M[k][k] - M[i][k] * M[k][j]) / prev
        prev = M[k][k]
    return sign * M[n - 1][n - 1]


def exact_inertia_by_minors(A, order):
    """Inertia from the signs of the leading principal minors (Jacobi's rule).

    Valid when no leading minor vanishes, which the test asserts.
    """
    Ap = [[A[i][j] for j in order] for i in order]
    n = len(Ap)
    prev = Fraction(1)
    neg = 0
    for k in range(1, n + 1):
        d = exact_det([row[:k] for row in Ap[:k]])
        assert d != 0, "a leading minor vanished; Jacobi's rule does not apply"
        if (d > 0) != (prev > 0):
            neg += 1
        prev = d
    return n - neg, 0, neg


def rel(x, y):
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    return float(np.abs(x - y).max() / max(np.abs(y).max(), 1e-300))


def tiny(N=3, nx=2, nu=1, seed=0):
    pat = kktgen.nmpc_pattern(N, nx, nu)
    vals = kktgen.dyadic_nmpc_values(pat, kktgen.rng_for(90, seed, 0))
    return pat, vals


# --------------------------------------------------------------------------
# generators and stored pattern statistics
# --------------------------------------------------------------------------

def test_generator_shapes():
    pat, v = kktgen.workload("small")
    assert (pat.n, pat.m, pat.nnz_j) == (450, 400, 1870)
    for rp, ci, nrow in ((pat.w_rowptr, pat.w_colind, pat.n), (pat.j_rowptr, pat.j_colind, pat.m)):
        assert len(rp) == nrow + 1 and rp[0] == 0 and (np.diff(rp) >= 0).all()
        for i in range(nrow):
            row = ci[rp[i]:rp[i + 1]]
            assert (np.diff(row) > 0).all()
    for i in range(pat.n):
        assert (pat.w_colind[pat.w_rowptr[i]:pat.w_rowptr[i + 1]] <= i).all()
    assert v.sigma_x.min() >= 1e-2 and v.sigma_x.max() <= 1e2
    # same seed -> same values; another value set -> different values
    _, v2 = kktgen.workload("small")
    _, v3 = kktgen.workload("small", value_set=1)
    assert np.array_equal(v.w_vals, v2.w_vals) and not np.array_equal(v.w_vals, v3.w_vals)


def test_paper_scale_shape():
    pat = kktgen.distillation_pattern(2000)
    assert (pat.n, pat.m) == (142000, 140000)
    assert pat.nnz_j == 66 + 2000 * 4 * 5 + 1999 * (62 * 6 + 4 * 4 + 66 * 4 + 66 + 66)


def test_golden_pattern_stats(oracle_lib):
    with open(os.path.join(HERE, "golden", "small_pattern_stats.json")) as fh:
        gold = json.load(fh)
    pat, v = kktgen.workload("small")
    K = Y.k_pattern(pat)
    st = Y.stats(Y.cholesky_structure(K))
    assert gold["nnz_j"] == pat.nnz_j
    assert gold["nnz_k_lower"] == (K.nnz + pat.n) // 2
    assert (st["nnz_l"], st["sum_c2"]) == (gold["nnz_l"], gold["sum_c2"]) == (4749, 50657)
    # second, independent route: the C oracle's elimination-tree column counts
    F = S.LDL(D.condensed(pat, v, v.sigma_s))
    cnt = F.colcounts() + 1
    assert int(cnt.sum()) == gold["nnz_l"] and int((cnt.astype(np.int64) ** 2).sum()) == gold["sum_c2"]
    assert np.array_equal(F.parent(), st["parent"])


# --------------------------------------------------------------------------
# exact rational ground truth
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(2, 2, 1), (3, 2, 1), (3, 3, 1)])
def test_exact_lifted(shape, oracle_lib):
    pat, v = tiny(*shape)
    A = D.lifted_saddle(pat, v)
    rhs = np.concatenate([v.b, np.zeros(pat.m)])
    xs = exact_solve(frac_matrix(A), rhs)
    x_exact = np.array([float(t) for t in xs[:pat.n]])
    # condensed K assembled exactly, solved exactly
    K = D.condensed(pat, v, v.sigma_s).toarray()
    x_cond = np.array([float(t) for t in exact_solve(frac_matrix(K), v.b)])
    assert np.array_equal(x_cond, x_exact)           # condensation is exact
    xb, inn = D.lifted_solution(pat, v, v.b)
    assert rel(xb, x_exact) < 1e-13
    xc, info = S.lifted_solve(pat, v, v.b)
    assert info["spd"] and rel(xc, x_exact) < 1e-14
    xs2, inn2, ok = S.lifted_saddle_solve(pat, v, v.b)
    assert ok and rel(xs2, x_exact) < 1e-13
    order = S.saddle_order(pat)
    exact_in = exact_inertia_by_minors(frac_matrix(A), order)
    assert exact_in == inn == inn2 == (pat.n, 0, pat.m)


@pytest.mark.parametrize("shape", [(2, 2, 1), (3, 2, 1)])
def test_exact_hykkt_gamma_independence(shape, oracle_lib):
    pat, v = tiny(*shape, seed=1)
    sols = []
    for gamma in (0.0, 4.0, 64.0):
        A = D.hykkt_saddle(pat, v, gamma)
        sols.append(exact_solve(frac_matrix(A), D.hykkt_rhs(pat, v, v.f, v.g, gamma)))
    assert sols[0] == sols[1] == sols[2]              # eq. (hykkt): exactly the same solution
    exact = np.array([float(t) for t in sols[0]])
    dx, dy, inn = D.hykkt_solution(pat, v, v.f, v.g, 0.0)
    assert rel(np.concatenate([dx, dy]), exact) < 1e-12
    dx2, dy2, inn2, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and rel(np.concatenate([dx2, dy2]), exact) < 1e-12
    exact_in = exact_inertia_by_minors(frac_matrix(D.hykkt_saddle(pat, v, 0.0)), S.saddle_order(pat))
    assert exact_in == inn == inn2 == (pat.n, 0, pat.m)


# --------------------------------------------------------------------------
# library brute force and paper identities at the small workload size
# --------------------------------------------------------------------------

def test_small_lifted_vs_numpy(oracle_lib):
    pat, v = kktgen.workload("small")
    K = D.condensed(pat, v, v.sigma_s)
    x_np = np.linalg.solve(K.toarray(), v.b)
    xb, inn = D.lifted_solution(pat, v, v.b)
    xc, info = S.lifted_solve(pat, v, v.b)
    assert inn == (pat.n, 0, pat.m) and info["spd"]
    assert D.forward_error(xb, x_np) < 1e-12 and D.forward_error(xc, x_np) < 1e-12
    be = D.backward_errors(K, xc, v.b)
    assert be["eta"] < 1e-15 and abs(be["eta"] - info["eta"]) <= 1e-3 * be["eta"] + 1e-30
    # scipy's LDL^T agrees on the inertia of the 2x2 form
    import scipy.linalg as sl
    _, dmat, _ = sl.ldl(D.lifted_saddle(pat, v))
    ev = np.linalg.eigvalsh(dmat)
    assert ((ev > 0).sum(), (ev < 0).sum()) == (pat.n, pat.m)


@pytest.mark.parametrize("n, m, dens, hubs", [(7, 3, 0.5, 0), (40, 30, 0.1, 0), (300, 200, 0.02, 2)])
def test_general_patterns_vs_numpy(oracle_lib, n, m, dens, hubs):
    """Unstructured patterns: the generator's W is symmetric positive definite
    with eigenvalues >= 1 (diagonal dominance), and the oracle's sparse LDL^T
    solve equals a dense solve of K to rounding."""
    pat = kktgen.general_pattern(kktgen.rng_for(5, n, 0), n, m, dens, hub_cols=hubs)
    v = kktgen.general_values(pat, kktgen.rng_for(5, n, 1), 1e-2, 1e2)
    rows = np.repeat(np.arange(n), np.diff(pat.w_rowptr))
    assert np.all(pat.w_colind <= rows) and np.all(np.isin(np.arange(n), pat.w_colind[pat.w_colind == rows]))
    W = sp.coo_matrix((v.w_vals, (rows, pat.w_colind)), shape=(n, n)).toarray()
    W = W + np.tril(W, -1).T
    assert np.linalg.eigvalsh(W).min() >= 1.0 - 1e-9
    K = D.condensed(pat, v, v.sigma_s)
    x_np = np.linalg.solve(K.toarray(), v.b)
    xc, info = S.lifted_solve(pat, v, v.b)
    assert info["spd"] and D.forward_error(xc, x_np) < 1e-12


def test_general_generator_structure():
    """The unstructured generator keeps its promises: with band > 0 every entry
    of W and J lies within the band, and with own_cols J has full row rank."""
    pat = kktgen.general_pattern(kktgen.rng_for(8, 0, 0), 2000, 1600, 0.3, row_max=6, band=40)
    rows = np.repeat(np.arange(pat.n), np.diff(pat.w_rowptr))
    assert np.all(rows - pat.w_colind <= 40) and np.all(pat.w_colind <= rows)
    for r in range(pat.m):
        c = pat.j_colind[pat.j_rowptr[r]:pat.j_rowptr[r + 1]]
        assert c.size == 0 or c.max() - c.min() < 40
    pat = kktgen.general_pattern(kktgen.rng_for(6, 2, 0), 300, 200, 0.02, hub_cols=2, own_cols=True)
    v = kktgen.general_values(pat, kktgen.rng_for(6, 2, 1), 1e-2, 1e2)
    J = sp.csr_matrix((v.j_vals, pat.j_colind, pat.j_rowptr), shape=(pat.m, pat.n)).toarray()
    assert np.linalg.matrix_rank(J) == pat.m


def test_condensation_identity():
    """Augmented 3x3 solve == condensed solve; slack steps recovered as stated."""
    pat, v = kktgen.workload("small", instance=1)
    rng = kktgen.rng_for(91, 0, 0)
    r1, r2, r4 = rng.standard_normal(pat.n), rng.standard_normal(pat.m), rng.standard_normal(pat.m)
    F = D.bunch_kaufman(D.lifted_augmented(pat, v))
    sol = F.solve(-np.concatenate([r1, r2, r4]))
    dx, ds, dz = sol[:pat.n], sol[pat.n:pat.n + pat.m], sol[pat.n + pat.m:]
    K = D.condensed(pat, v, v.sigma_s).toarray()
    dx_c = np.linalg.solve(K, D.condensed_rhs(pat, v, r1, r2, r4))
    assert D.forward_error(dx, dx_c) < 1e-11
    ds_c, dz_c = D.recover_slack_steps(pat, v, dx_c, r2, r4)
    assert D.forward_error(ds, ds_c) < 1e-10 and D.forward_error(dz, dz_c) < 1e-10
    assert F.inertia() == (pat.n + pat.m, 0, pat.m)


def test_gamma_independence_float(oracle_lib):
    pat, v = kktgen.workload("hykkt")
    dx0, dy0, inn0, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and inn0 == (pat.n, 0, pat.m)
    for gamma, tol in ((1e4, 1e-11), (1e6, 1e-10), (1e8, 1e-8)):
        dx, dy, inn = D.hykkt_solution(pat, v, v.f, v.g, gamma)
        assert inn == (pat.n, 0, pat.m)
        assert D.forward_error(dx, dx0) < tol
        dxc, dyc, info = S.hykkt_cg_solve(pat, v, v.f, v.g, gamma, tol=1e-10)
        assert info["status"] == "ok" and D.forward_error(dxc, dx0) < tol
        assert D.hykkt_backward_errors(pat, v, dxc, dyc, v.f, v.g)["eta"] < 1e-10


def test_haynsworth_and_planted_indefinite(oracle_lib):
    pat, v = kktgen.workload("small", instance=2)
    F = S.LDL(D.condensed(pat, v, v.sigma_s))
    assert F.ok and (F.d() > 0).all()
    assert D.bunch_kaufman(D.lifted_saddle(pat, v)).inertia() == (pat.n, 0, pat.m)
    assert D.bunch_kaufman(D.lifted_augmented(pat, v)).inertia() == (pat.n + pat.m, 0, pat.m)
    # make K indefinite: a large negative primal diagonal on one stage
    s = pat.meta["stage"]
    k0 = 20 * s
    v.sigma_x[k0:k0 + s] = -1e4
    x, info = S.lifted_solve(pat, v, v.b)
    assert not info["spd"] and x is None and k0 <= info["bad_col"] < k0 + s
    eig = np.linalg.eigvalsh(D.condensed(pat, v, v.sigma_s).toarray())
    assert eig.min() < 0
    assert D.bunch_kaufman(D.lifted_saddle(pat, v)).inertia() != (pat.n, 0, pat.m)
    assert D.bunch_kaufman(D.lifted_augmented(pat, v)).inertia() != (pat.n + pat.m, 0, pat.m)


def test_schur_closed_form_and_cg_counts(oracle_lib):
    pat, v = kktgen.workload("hykkt")
    s0 = np.linalg.eigvalsh(D.schur_dense(pat, v, 0.0))
    assert s0.min() > 0
    counts = {}
    for gamma in (1e4, 1e6, 1e7, 1e8):
        sg = np.linalg.eigvalsh(D.schur_dense(pat, v, gamma))
        pred = np.sort(D.schur_eigs_closed_form(s0, gamma))
        assert np.abs(sg - pred).max() <= 1e-6 / gamma
        assert abs(sg.mean() * gamma - 1.0) < 1.0 / (gamma * s0.min())
        kappa = pred.max() / pred.min()
        _, _, info = S.hykkt_cg_solve(pat, v, v.f, v.g, gamma, tol=1e-10)
        assert info["status"] == "ok"
        assert info["iters"] <= D.cg_iteration_bound(kappa, 1e-10)
        counts[gamma] = info["iters"]
    assert counts[1e7] < 10                        # fewer than 10 iterations at gamma = 1e7
    assert counts[1e4] >= counts[1e6] >= counts[1e8]


# --------------------------------------------------------------------------
# special cases that reduce to textbook routines
# --------------------------------------------------------------------------

def thomas(a, b, c, d):
    """Tridiagonal solve: sub-diagonal a[1:], diagonal b, super-diagonal c[:-1]."""
    n = len(b)
    cp, dp = np.zeros(n), np.zeros(n)
    cp[0], dp[0] = c[0] / b[0], d[0] / b[0]
    for i in range(1, n):
        den = b[i] - a[i] * cp[i - 1]
        cp[i] = c[i] / den if i < n - 1 else 0.0
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den
    x = np.zeros(n)
    x[-1] = dp[-1]
    for i in range(n - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def test_scalar_chain_is_tridiagonal(oracle_lib):
    pat = kktgen.nmpc_pattern(40, 1, 0)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(92, 0, 0), 1e-2, 1e2)
    K = D.condensed(pat, v, v.sigma_s).toarray()
    assert np.count_nonzero(np.triu(K, 2)) == 0
    x_t = thomas(np.r_[0, np.diag(K, -1)], np.diag(K).copy(), np.r_[np.diag(K, 1), 0], v.b)
    xc, info = S.lifted_solve(pat, v, v.b)
    xb, _ = D.lifted_solution(pat, v, v.b)
    assert D.forward_error(xc, x_t) < 1e-13 and D.forward_error(xb, x_t) < 1e-12


def test_single_stage_is_dense_cholesky(oracle_lib):
    pat = kktgen.nmpc_pattern(1, 6, 2)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(92, 1, 0), 1e-2, 1e2)
    K = D.condensed(pat, v, v.sigma_s).toarray()
    Lc = np.linalg.cholesky(K)
    x_ref = np.linalg.solve(Lc.T, np.linalg.solve(Lc, v.b))
    xc, info = S.lifted_solve(pat, v, v.b)
    assert D.forward_error(xc, x_ref) < 1e-13
    F = S.LDL(K)
    assert np.allclose(np.sqrt(F.d()), np.diag(Lc), rtol=1e-12)


def test_no_constraints_is_plain_cholesky(oracle_lib):
    pat = kktgen.nmpc_pattern(5, 3, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(92, 2, 0), 1e-2, 1e2)
    empty = kktgen.Pattern(pat.n, 0, pat.w_rowptr, pat.w_colind, np.zeros(1, np.int32),
                           np.zeros(0, np.int32), pat.meta)
    ve = kktgen.Values(v.w_vals, np.zeros(0), v.sigma_x, np.zeros(0), v.b, v.f, np.zeros(0))
    K = D.condensed(empty, ve, ve.sigma_s).toarray()
    Lc = np.linalg.cholesky(K)
    xc, info = S.lifted_solve(empty, ve, ve.b)
    assert D.forward_error(xc, np.linalg.solve(Lc.T, np.linalg.solve(Lc, ve.b))) < 1e-13


def test_gamma_zero_is_range_space(oracle_lib):
    pat = kktgen.nmpc_pattern(6, 3, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(92, 3, 0), 1e-1, 1e1)
    dx0, dy0, _ = D.hykkt_solution(pat, v, v.f, v.g, 0.0)
    dx, dy, info = S.hykkt_cg_solve(pat, v, v.f, v.g, 0.0, tol=1e-12, maxit=500)
    assert info["status"] == "ok"
    # range-space method: dy = (J K0^{-1} J^T)^{-1} (J K0^{-1} f - g), dx = K0^{-1}(f - J^T dy)
    K0 = D.condensed(pat, v, 0.0).toarray()
    J = D.jacobian(pat, v).toarray()
    Sm = J @ np.linalg.solve(K0, J.T)
    dy_r = np.linalg.solve(Sm, J @ np.linalg.solve(K0, v.f) - v.g)
    dx_r = np.linalg.solve(K0, v.f - J.T @ dy_r)
    assert D.forward_error(dx, dx_r) < 1e-9 and D.forward_error(dx0, dx_r) < 1e-10
    assert D.forward_error(dy, dy_r) < 1e-9


def test_refinement_ill_conditioned(oracle_lib):
    """Sigma over 16 decades: refinement drives omega to O(u), eta below the 1e-10 gate."""
    pat, _ = kktgen.small_config()
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 7, 0), 1e-8, 1e8)
    K = D.condensed(pat, v, v.sigma_s)
    xc, info = S.lifted_solve(pat, v, v.b)
    be = D.backward_errors(K, xc, v.b)
    assert be["eta"] <= 1e-15 and be["omega"] <= 1e-14 * 10
    xb, _ = D.lifted_solution(pat, v, v.b)
    cond = np.linalg.cond(K.toarray())
    assert D.forward_error(xc, xb) <= 1e-15 * cond * 10


# --------------------------------------------------------------------------
# planted mistakes must be caught
# --------------------------------------------------------------------------

def test_planted_mistakes_are_caught(monkeypatch, oracle_lib):
    def fails(check):
        try:
            check()
        except AssertionError:
            return True
        return False

    # 1) a dropped term: Sigma_x missing from the condensed matrix
    orig = D.condensed
    monkeypatch.setattr(D, "condensed", lambda p, v, d: orig(p, v, d) - sp.diags(v.sigma_x))
    assert fails(test_condensation_identity)
    monkeypatch.setattr(D, "condensed", orig)

    # 2) a wrong sign in the slack recovery
    orig_rec = D.recover_slack_steps
    monkeypatch.setattr(D, "recover_slack_steps",
                        lambda p, v, dx, r2, r4: tuple(-t for t in orig_rec(p, v, dx, r2, r4)))
    assert fails(test_condensation_identity)
    monkeypatch.setattr(D, "recover_slack_steps", orig_rec)

    # 3) the gamma J^T g shift dropped from the HyKKT right-hand side
    monkeypatch.setattr(D, "hykkt_rhs", lambda p, v, f, g, gamma: np.concatenate([f, g]))
    assert fails(lambda: test_exact_hykkt_gamma_independence((2, 2, 1), None))
    monkeypatch.undo()

    # 4) a transposed operand: J instead of J^T in the saddle-point block
    orig_saddle = D.lifted_saddle

    def bad_saddle(p, v):
        A = orig_saddle(p, v).copy()
        n = p.n
        A[:n, n:] = np.roll(A[:n, n:], 1, axis=0)
        return A
    monkeypatch.setattr(D, "lifted_saddle", bad_saddle)
    assert fails(lambda: test_exact_lifted((2, 2, 1), None))
    monkeypatch.undo()


# --------------------------------------------------------------------------
# the evaluators: backward errors by hand and by their defining perturbations
# --------------------------------------------------------------------------

def test_backward_errors_hand_computed():
    """eta, omega and relres of a 3x3 system, worked out by hand.

    A = [[4,-1,0],[-1,4,-1],[0,-1,4]], x = [1,-2,1/2], b = [13/2,-19/2,3]:
    A x = [6, -19/2, 4], so r = b - A x = [1/2, 0, -1].
    ||A||_inf = 6 (middle row), ||x||_inf = 2, ||b||_inf = 19/2:
      eta = 1 / (6*2 + 19/2) = 2/43.
    |A||x| = [6, 19/2, 4], |A||x| + |b| = [25/2, 19, 7]:
      omega = max(1/25, 0, 1/7) = 1/7;   relres = 1 / (19/2) = 2/19.
    """
    A = np.array([[4.0, -1.0, 0.0], [-1.0, 4.0, -1.0], [0.0, -1.0, 4.0]])
    x = np.array([1.0, -2.0, 0.5])
    b = np.array([6.5, -9.5, 3.0])
    for M in (A, sp.csr_matrix(A)):
        be = D.backward_errors(M, x, b)
        assert be["eta"] == pytest.approx(2.0 / 43.0, rel=1e-15)
        assert be["omega"] == pytest.approx(1.0 / 7.0, rel=1e-15)
        assert be["relres"] == pytest.approx(2.0 / 19.0, rel=1e-15)
    # an exact solution has zero backward error; 0/0 rows count as zero
    be = D.backward_errors(A, np.zeros(3), np.zeros(3))
    assert be == dict(eta=0.0, omega=0.0, relres=0.0)


def test_backward_errors_attained_by_perturbations():
    """The two backward errors are the sizes of perturbations that make x exact.

    Rigal-Gaches: with z = sign(x_k) e_k (k the largest |x_k|) and
    t = 1 / (||A|| ||x|| + ||b||), the system (A + ||A|| t r z^T) x = b - ||b|| t r
    holds exactly, with ||dA|| = eta ||A|| and ||db|| = eta ||b||.
    Oettli-Prager: with s_i = r_i / (|A||x| + |b|)_i, the rows
    dA = diag(s) |A| diag(sign x), db = -diag(s) |b| make x exact, with
    |dA| <= omega |A| and |db| <= omega |b|. Any smaller perturbation leaves a
    residual, since ||r|| <= eps (||A|| ||x|| + ||b||) (normwise) and
    |r| <= eps (|A||x| + |b|) (componentwise) for a perturbation of size eps.
    """
    rng = np.random.default_rng(11)
    A = rng.standard_normal((7, 7))
    x = rng.standard_normal(7)
    b = A @ x + 1e-3 * rng.standard_normal(7)
    be = D.backward_errors(A, x, b)
    r = b - A @ x
    nA = np.abs(A).sum(axis=1).max()
    k = int(np.argmax(np.abs(x)))
    z = np.zeros(7)
    z[k] = np.sign(x[k])
    t = 1.0 / (nA * np.abs(x).max() + np.abs(b).max())
    dA = nA * t * np.outer(r, z)
    db = -np.abs(b).max() * t * r
    assert np.abs((A + dA) @ x - (b + db)).max() <= 1e-14 * np.abs(b).max()
    assert np.abs(dA).sum(axis=1).max() == pytest.approx(be["eta"] * nA, rel=1e-12)
    assert np.abs(db).max() == pytest.approx(be["eta"] * np.abs(b).max(), rel=1e-12)
    s = r / (np.abs(A) @ np.abs(x) + np.abs(b))
    dA = s[:, None] * np.abs(A) * np.sign(x)[None, :]
    db = -s * np.abs(b)
    assert np.abs((A + dA) @ x - (b + db)).max() <= 1e-14 * np.abs(b).max()
    assert np.abs(s).max() == pytest.approx(be["omega"], rel=1e-12)
    assert (np.abs(dA) <= be["omega"] * np.abs(A) * (1 + 1e-12)).all()


def test_componentwise_error_hand_computed():
    """x* = [1000, -2, 1e-9], x = [1000.001, -2, 2e-9], floor 1e-12:
    entry errors 1e-3 / (1000 + 1e-9), 0, 1e-9 / (1e-9 + 1e-9) = 1/2."""
    xs = np.array([1000.0, -2.0, 1e-9])
    x = np.array([1000.001, -2.0, 2e-9])
    assert D.componentwise_error(x, xs) == pytest.approx(0.5, rel=1e-9)
    assert D.componentwise_error(x[:2], xs[:2]) == pytest.approx(1e-6, rel=1e-6)
    assert D.componentwise_error(xs, xs) == 0.0


def test_oracle_routes_agree_componentwise(oracle_lib):
    """Three independent routes to the Lifted-KKT x* (Bunch-Kaufman on the 2x2
    form, the C sparse LDL^T with refinement, numpy's LU of K) and two to the
    HyKKT (dx*, dy*) agree entry by entry, not only in norm, on the
    well-conditioned small workload."""
    pat, v = kktgen.workload("small")
    xb, _ = D.lifted_solution(pat, v, v.b)
    xc, info = S.lifted_solve(pat, v, v.b)
    xn = np.linalg.solve(D.condensed(pat, v, v.sigma_s).toarray(), v.b)
    assert D.componentwise_error(xb, xn) <= 1e-11 and D.componentwise_error(xc, xn) <= 1e-11
    pat, v = kktgen.workload("hykkt")
    dxb, dyb, _ = D.hykkt_solution(pat, v, v.f, v.g, 0.0)
    dxs, dys, _, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok
    assert D.componentwise_error(dxs, dxb) <= 1e-10 and D.componentwise_error(dys, dyb) <= 1e-10


def test_hykkt_wide_sigma_small_system(oracle_lib):
    """The small NMPC system with Sigma_x ~ logU[1e-8, 1e8] (late-iteration
    range) at gamma = 1e7: the Schur CG converges within the closed-form bound,
    and its (dx, dy) agrees with Bunch-Kaufman on the saddle system although
    that system's condition number is ~1e15, because the perturbations the
    wide Sigma_x causes are diagonal scalings the two methods both absorb."""
    pat, _ = kktgen.small_config()
    v = kktgen.nmpc_values(pat, kktgen.rng_for(2, 0, 9), 1e-8, 1e8)
    K0 = D.condensed(pat, v, 0.0).toarray()
    J = D.jacobian(pat, v).toarray()
    s0 = np.linalg.eigvalsh(J @ np.linalg.solve(K0, J.T))
    e = D.schur_eigs_closed_form(s0, 1e7)
    dxb, dyb, inn = D.hykkt_solution(pat, v, v.f, v.g, 0.0)
    assert inn == (pat.n, 0, pat.m)
    dx, dy, info = S.hykkt_cg_solve(pat, v, v.f, v.g, 1e7, tol=1e-10, maxit=1000)
    assert info["status"] == "ok" and info["iters"] <= D.cg_iteration_bound(e.max() / e.min(), 1e-10)
    assert D.hykkt_backward_errors(pat, v, dx, dy, v.f, v.g)["eta"] <= 1e-10
    assert D.forward_error(dx, dxb) <= 1e-7 and D.forward_error(dy, dyb) <= 1e-7


def test_inertia_correction_rule():
    """The oracle's inertia correction (delta raised until the regularised
    augmented system has the inertia of eq. (inertia)) against the spectrum of
    the condensed matrix: by Haynsworth's formula (stated after eq.
    (kkt:condensed)) the augmented inertia is right exactly when K + delta I
    is positive definite, so the accepted delta is the first trial with
    lambda_min(K + delta I) > 0 and every earlier trial has lambda_min <= 0.
    The trials follow the update rule: delta_first, then factors of
    kappa_plus_first; with an earlier success, kappa_minus * delta_last, then
    factors of kappa_plus."""
    pat = kktgen.nmpc_pattern(10, 4, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(95, 0, 0), 1e-2, 1e2)
    K = D.condensed(pat, v, v.sigma_s).toarray()
    assert D.inertia_correction(pat, v) == (0.0, [0.0], 0.0)   # already positive definite
    s = pat.meta["stage"]
    v.sigma_x[3 * s:4 * s] -= 30.0 + np.linalg.eigvalsh(K).max()
    K = D.condensed(pat, v, v.sigma_s).toarray()
    lmin = np.linalg.eigvalsh(K).min()
    assert lmin < -30.0
    delta, trials, last = D.inertia_correction(pat, v)
    assert trials[:2] == [0.0, 1e-4] and len(trials) >= 5   # lambda_min < -30 needs delta > 30
    for a, b in zip(trials[1:], trials[2:]):
        assert b == pytest.approx(100.0 * a, rel=1e-15)
    assert delta == trials[-1] == last
    assert np.linalg.eigvalsh(K + delta * np.eye(pat.n)).min() > 0
    for t in trials[:-1]:
        assert np.linalg.eigvalsh(K + t * np.eye(pat.n)).min() <= 0
    # an earlier success: start from kappa_minus * delta_last, grow by kappa_plus
    delta2, trials2, last2 = D.inertia_correction(pat, v, delta_last=delta)
    assert trials2[1] == pytest.approx(delta / 3.0, rel=1e-15)
    for a, b in zip(trials2[1:], trials2[2:]):
        assert b == pytest.approx(8.0 * a, rel=1e-15)
    assert np.linalg.eigvalsh(K + delta2 * np.eye(pat.n)).min() > 0
    for t in trials2[:-1]:
        assert np.linalg.eigvalsh(K + t * np.eye(pat.n)).min() <= 0
    # beyond delta_max: no delta
    assert D.inertia_correction(pat, v, delta_max=1.0)[0] is None


def test_general_hykkt_condensation_and_gamma_independence():
    """Equality rows G and inequality rows H: the augmented system of eq.
    (kkt:augmented) with both, condensed as in eq. (kkt:condensed), gives the
    saddle system [[K_k, G^T], [G, 0]] with K_k = W + Sigma_x + H^T D_s H and
    right-hand side -[r1 + H^T (D_s r4 - r2); r3]; adding gamma G^T G with the
    shifted right-hand side (eq. (hykkt), r_gamma) leaves (d_x, d_y) unchanged.
    Checked with numpy's solver on the explicit matrices; the inertia of the
    augmented system is (n + m_i, 0, m_i + m_e) (eq. (inertia))."""
    pat, v = kktgen.workload("small", instance=3)
    eq = np.arange(0, pat.m, 2)          # every other row an equality
    G, H, ds, eqi, ineq = D.split_rows(pat, v, eq)
    n, me, mi = pat.n, len(eqi), len(ineq)
    rng = kktgen.rng_for(97, 0, 0)
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    A = D.general_augmented(pat, v, eq)
    z = np.linalg.solve(A, -np.concatenate([r1, r2, r3, r4]))
    dx, dsv, dy, dz = z[:n], z[n:n + mi], z[n + mi:n + mi + me], z[n + mi + me:]
    ev = np.linalg.eigvalsh(A)
    assert ((ev > 0).sum(), (ev == 0).sum(), (ev < 0).sum()) == (n + mi, 0, mi + me)
    f = -(r1 + H.T @ (ds * r4 - r2))
    g = -r3
    for gamma in (0.0, 1e2, 1e4):
        S = D.general_hykkt_saddle(pat, v, eq, gamma)
        sol = np.linalg.solve(S, np.concatenate([f + gamma * (G.T @ g), g]))
        assert D.forward_error(sol[:n], dx) < 1e-9 and D.forward_error(sol[n:], dy) < 1e-9, gamma
    # slack and multiplier recovery with the inequality rows
    assert D.forward_error(dsv, -r4 - H @ dx) < 1e-10
    assert D.forward_error(dz, -r2 - ds * dsv) < 1e-10


def test_qp_ipm_kkt_certificate_and_slsqp():
    """The oracle's interior-point method on a convex QP (section
    "INTERIOR-POINT METHOD"): its answer satisfies the QP's KKT conditions
    (stationarity, primal feasibility, z >= 0, complementarity) to the
    tolerance, and on a tiny instance matches scipy's SLSQP solution of the
    same QP (an active-set method, independent of the IPM)."""
    from scipy.optimize import minimize
    from oracle import ipm
    pat = kktgen.nmpc_pattern(4, 2, 1)          # n = 12, m = 8
    v = kktgen.nmpc_values(pat, kktgen.rng_for(99, 0, 0), 1e-2, 1e2)
    rng = kktgen.rng_for(99, 1, 0)
    c = rng.standard_normal(pat.n)
    u = 0.1 + 0.5 * rng.random(pat.m)
    W, c, J, u = ipm.qp_from_pattern(pat, v, c, u)
    x, s, z, info = ipm.qp_ipm(W, c, J, u, np.zeros(pat.n), u.copy(), np.ones(pat.m), tol=1e-10)
    assert info["status"] == "ok", info
    Wd, Jd = W.toarray(), J.toarray()
    assert np.abs(Wd @ x + c + Jd.T @ z).max() <= 1e-8
    assert (Jd @ x - u).max() <= 1e-9 and z.min() > 0 and s.min() > 0
    assert abs(s @ z) <= 1e-8 * pat.m
    active = (z > 1e-6).sum()
    assert 0 < active < pat.m                    # some constraints bind, some do not
    res = minimize(lambda y: 0.5 * y @ Wd @ y + c @ y, np.zeros(pat.n), jac=lambda y: Wd @ y + c,
                   constraints=[dict(type="ineq", fun=lambda y: u - Jd @ y, jac=lambda y: -Jd)],
                   method="SLSQP", options=dict(ftol=1e-14, maxiter=500))
    assert res.success
    assert np.abs(res.x - x).max() <= 1e-6 * (1 + np.abs(x).max())
