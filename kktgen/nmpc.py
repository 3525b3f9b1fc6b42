"""Pattern and value generators for dynamic (NMPC-shaped) KKT systems.

Variables are stored stage-major. Stage k owns z_k = (x_k, [a_k,] u_k):
x_k are the states, a_k the algebraic variables (distillation shape only),
u_k the controls. The Jacobian J stacks the initial-state rows and, for
every step k, the dynamics rows x_{k+1} - A_k x_k - C_k a_k - B_k u_k (and
the algebraic rows of the distillation shape). The Hessian W is block
diagonal with one symmetric positive definite block per stage.

Patterns are returned as 0-based int32 CSR arrays: W as its lower triangle
(col <= row), J as an m x n matrix, both with sorted, duplicate-free
columns. Values are float64 arrays in the same entry order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

SEED_ROOT = 240315913


def rng_for(config: int, instance: int = 0, value_set: int = 0) -> np.random.Generator:
    """Independent, reproducible stream for one (config, instance, value set)."""
    return np.random.default_rng(np.random.SeedSequence([SEED_ROOT, config, instance, value_set]))


def log_uniform(rng: np.random.Generator, lo: float, hi: float, size) -> np.ndarray:
    """exp(U(ln lo, ln hi)) samples."""
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


@dataclass
class Pattern:
    n: int
    m: int
    w_rowptr: np.ndarray
    w_colind: np.ndarray
    j_rowptr: np.ndarray
    j_colind: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def nnz_w(self) -> int:
        return int(self.w_rowptr[-1])

    @property
    def nnz_j(self) -> int:
        return int(self.j_rowptr[-1])


@dataclass
class Values:
    w_vals: np.ndarray
    j_vals: np.ndarray
    sigma_x: np.ndarray
    sigma_s: np.ndarray
    b: np.ndarray       # right-hand side of the condensed (Lifted) system, length n
    f: np.ndarray       # primal right-hand side of the saddle-point system, length n
    g: np.ndarray       # dual right-hand side of the saddle-point system, length m


def _csr_from_rows(rows: list, ncols: int):
    """rows: list of sorted int arrays of column indices -> (rowptr, colind)."""
    lens = np.fromiter((len(r) for r in rows), dtype=np.int64, count=len(rows))
    rowptr = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    colind = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    assert rowptr[-1] < 2**31
    return rowptr.astype(np.int32), colind


# --------------------------------------------------------------------------
# NMPC shape: z_k = (x_k, u_k), tridiagonal A_k, dense B_k, dense SPD W_k
# --------------------------------------------------------------------------

def _tridiag_cols(i: int, nx: int) -> np.ndarray:
    return np.arange(max(0, i - 1), min(nx, i + 2))


def nmpc_pattern(N: int, nx: int, nu: int) -> Pattern:
    s = nx + nu
    n = N * s
    m = N * nx
    # W: dense lower triangle of each s x s stage block.
    w_rows = []
    for k in range(N):
        base = k * s
        for r in range(s):
            w_rows.append(np.arange(base, base + r + 1))
    # J: initial rows, then nx dynamics rows per step k = 0..N-2.
    j_rows = [np.array([i]) for i in range(nx)]
    for k in range(N - 1):
        xk, uk, xk1 = k * s, k * s + nx, (k + 1) * s
        for i in range(nx):
            j_rows.append(np.concatenate([xk + _tridiag_cols(i, nx), uk + np.arange(nu), [xk1 + i]]))
    wr, wc = _csr_from_rows(w_rows, n)
    jr, jc = _csr_from_rows(j_rows, n)
    return Pattern(n, m, wr, wc, jr, jc,
                   dict(kind="nmpc", N=N, nx=nx, nu=nu, stage=s))


def _stage_dense_lower(Wk: np.ndarray) -> np.ndarray:
    s = Wk.shape[0]
    return np.concatenate([Wk[r, :r + 1] for r in range(s)])


def nmpc_values(pat: Pattern, rng: np.random.Generator, sigma_lo: float, sigma_hi: float) -> Values:
    """Draw order: per stage W_k (M ~ N(0,1)), then per step A_k, B_k, then Σx, Σs, b, f, g."""
    N, nx, nu = pat.meta["N"], pat.meta["nx"], pat.meta["nu"]
    s = nx + nu
    w_parts = []
    for _ in range(N):
        M = rng.standard_normal((s, s))
        w_parts.append(_stage_dense_lower(M @ M.T + 0.1 * np.eye(s)))
    j_parts = [np.ones(nx)]
    for _ in range(N - 1):
        # tridiagonal A_k: U(-0.5, 0.5) entries plus 0.9 on the diagonal
        A = np.zeros((nx, nx))
        for i in range(nx):
            cols = _tridiag_cols(i, nx)
            A[i, cols] = rng.uniform(-0.5, 0.5, len(cols))
            A[i, i] += 0.9
        B = rng.standard_normal((nx, nu))
        for i in range(nx):
            j_parts.append(np.concatenate([-A[i, _tridiag_cols(i, nx)], -B[i], [1.0]]))
    w_vals = np.concatenate(w_parts)
    j_vals = np.concatenate(j_parts)
    assert len(w_vals) == pat.nnz_w and len(j_vals) == pat.nnz_j
    return Values(w_vals, j_vals,
                  log_uniform(rng, sigma_lo, sigma_hi, pat.n),
                  log_uniform(rng, sigma_lo, sigma_hi, pat.m),
                  rng.standard_normal(pat.n), rng.standard_normal(pat.n), rng.standard_normal(pat.m))


def dyadic_nmpc_values(pat: Pattern, rng: np.random.Generator) -> Values:
    """NMPC values that are exact binary fractions (and whose products stay exact).

    Entries of M, A, B, the right-hand sides and Σ are small multiples of
    powers of two, so float64 holds every input exactly and an exact
    rational computation sees the same numbers.
    """
    N, nx, nu = pat.meta["N"], pat.meta["nx"], pat.meta["nu"]
    s = nx + nu
    halves = np.array([-1.0, -0.5, 0.5, 1.0])
    w_parts = []
    for _ in range(N):
        M = rng.choice(halves, size=(s, s))
        w_parts.append(_stage_dense_lower(M @ M.T + 0.125 * np.eye(s)))
    j_parts = [np.ones(nx)]
    for _ in range(N - 1):
        for i in range(nx):
            a = rng.choice(halves, size=len(_tridiag_cols(i, nx)))
            bcol = rng.choice(halves, size=nu)
            j_parts.append(np.concatenate([-a, -bcol, [1.0]]))
    pw = np.array([0.25, 0.5, 1.0, 2.0, 4.0])
    return Values(np.concatenate(w_parts), np.concatenate(j_parts),
                  rng.choice(pw, pat.n), rng.choice(pw, pat.m),
                  rng.choice(halves, pat.n), rng.choice(halves, pat.n), rng.choice(halves, pat.m))


# --------------------------------------------------------------------------
# Distillation-column shape: z_k = (x_k [33 two-tray blocks], a_k [4], u_k [1])
# --------------------------------------------------------------------------

def _blocktri_cols(i: int, nx: int) -> np.ndarray:
    b = i // 2
    nb = nx // 2
    lo, hi = max(0, b - 1), min(nb - 1, b + 1)
    return np.arange(2 * lo, 2 * hi + 2)


def distillation_pattern(N: int, nx: int = 66, na: int = 4, nu: int = 1) -> Pattern:
    assert nx % 2 == 0
    s = nx + na + nu
    n = N * s
    # W_k pentadiagonal: lower pattern j in [i-2, i] within the stage
    w_rows = []
    for k in range(N):
        base = k * s
        for r in range(s):
            w_rows.append(np.arange(base + max(0, r - 2), base + r + 1))
    j_rows = [np.array([i]) for i in range(nx)]
    for k in range(N):
        xk, ak, uk = k * s, k * s + nx, k * s + nx + na
        alg = np.concatenate([ak + np.arange(na), uk + np.arange(nu)])
        for _ in range(na):
            j_rows.append(alg)
        if k <= N - 2:
            xk1 = (k + 1) * s
            for i in range(nx):
                j_rows.append(np.concatenate([xk + _blocktri_cols(i, nx), alg, [xk1 + i]]))
    wr, wc = _csr_from_rows(w_rows, n)
    jr, jc = _csr_from_rows(j_rows, n)
    m = len(j_rows)
    return Pattern(n, m, wr, wc, jr, jc,
                   dict(kind="distillation", N=N, nx=nx, na=na, nu=nu, stage=s))


def distillation_values(pat: Pattern, rng: np.random.Generator, sigma_lo: float, sigma_hi: float) -> Values:
    """Draw order: per stage W_k (banded M), per stage F_k, g_k, A_k, C_k, B_k; then Σx, Σs, b, f, g."""
    N, nx, na, nu = pat.meta["N"], pat.meta["nx"], pat.meta["na"], pat.meta["nu"]
    s = nx + na + nu
    w_parts = []
    for _ in range(N):
        M = np.zeros((s, s))
        for d in range(3):
            idx = np.arange(d, s)
            M[idx, idx - d] = rng.standard_normal(s - d)
        Wk = M @ M.T + 0.1 * np.eye(s)
        w_parts.append(np.concatenate([Wk[r, max(0, r - 2):r + 1] for r in range(s)]))
    j_parts = [np.ones(nx)]
    for k in range(N):
        F = np.eye(na) + 0.25 * rng.uniform(-1, 1, (na, na)) * (1 - np.eye(na))
        gk = rng.uniform(-1, 1, (na, nu))
        for r in range(na):
            j_parts.append(np.concatenate([F[r], gk[r]]))
        if k <= N - 2:
            for i in range(nx):
                cols = _blocktri_cols(i, nx)
                a = rng.uniform(-1, 1, len(cols))
                c = rng.uniform(-1, 1, na)
                bb = rng.uniform(-1, 1, nu)
                j_parts.append(np.concatenate([-a, -c, -bb, [1.0]]))
    w_vals = np.concatenate(w_parts)
    j_vals = np.concatenate(j_parts)
    assert len(w_vals) == pat.nnz_w and len(j_vals) == pat.nnz_j
    return Values(w_vals, j_vals,
                  log_uniform(rng, sigma_lo, sigma_hi, pat.n),
                  log_uniform(rng, sigma_lo, sigma_hi, pat.m),
                  rng.standard_normal(pat.n), rng.standard_normal(pat.n), rng.standard_normal(pat.m))


# --------------------------------------------------------------------------
# Workload recipes (sizes and Σ ranges of the benchmark configurations)
# --------------------------------------------------------------------------

def hub_pattern(k: int, b: int, h1: int, h2: int) -> Pattern:
    """k independent branches of b variables, each coupled to a hub of h1
    variables, which is coupled to a root block of h2 (variables numbered
    branch by branch, then the hub, then the root). W: a dense lower block
    per branch, hub and root. J: per branch two rows on the branch and the
    hub; two rows on the hub and the root. In the natural order the hub's
    supernode has k children."""
    n = k * b + h1 + h2
    hub0, root0 = k * b, k * b + h1
    w_rows = []
    for base, s in [(i * b, b) for i in range(k)] + [(hub0, h1), (root0, h2)]:
        for r in range(s):
            w_rows.append(np.arange(base, base + r + 1))
    j_rows = []
    for i in range(k):
        for _ in range(2):
            j_rows.append(np.concatenate([np.arange(i * b, (i + 1) * b), np.arange(hub0, hub0 + h1)]))
    for _ in range(2):
        j_rows.append(np.arange(hub0, n))
    wr, wc = _csr_from_rows(w_rows, n)
    jr, jc = _csr_from_rows(j_rows, n)
    return Pattern(n, len(j_rows), wr, wc, jr, jc, dict(kind="hub", k=k, b=b, h1=h1, h2=h2))


def hub_values(pat: Pattern, rng: np.random.Generator, sigma_lo: float, sigma_hi: float) -> Values:
    """Draw order: per block W (M ~ N(0,1), M M^T + I), then J ~ N(0,1), then Σx, Σs, b, f, g."""
    k, b, h1, h2 = (pat.meta[x] for x in ("k", "b", "h1", "h2"))
    w_parts = []
    for s in [b] * k + [h1, h2]:
        M = rng.standard_normal((s, s))
        w_parts.append(_stage_dense_lower(M @ M.T + np.eye(s)))
    w_vals = np.concatenate(w_parts)
    j_vals = rng.standard_normal(pat.nnz_j)
    assert len(w_vals) == pat.nnz_w
    return Values(w_vals, j_vals,
                  log_uniform(rng, sigma_lo, sigma_hi, pat.n),
                  log_uniform(rng, sigma_lo, sigma_hi, pat.m),
                  rng.standard_normal(pat.n), rng.standard_normal(pat.n), rng.standard_normal(pat.m))


# --------------------------------------------------------------------------
# general sparse patterns (no stage structure)
# --------------------------------------------------------------------------

def general_pattern(rng: np.random.Generator, n: int, m: int, density: float, row_max: int = 5,
                    hub_cols: int = 0, hub_frac: float = 0.5, own_cols: bool = False, band: int = 0) -> Pattern:
    """Unstructured pattern: W's row i holds its diagonal and each earlier
    column with probability `density`; J's rows hold 0 .. row_max random
    columns, plus each of the last `hub_cols` columns with probability
    `hub_frac` (columns shared by many rows: entries of J^T J with long
    product lists). With own_cols (m <= n), row r also holds column q_r of
    a random permutation q, so J has full row rank for random values. With
    band > 0 every entry lies within `band` of the diagonal (W's row i draws
    from columns i-band .. i-1, J's row from a window of width band at a
    random place), as on a one-dimensional mesh."""
    w_rows = []
    for i in range(n):
        lo = max(0, i - band) if band else 0
        lower = lo + np.flatnonzero(rng.random(i - lo) < density) if i > lo else np.zeros(0, np.int64)
        w_rows.append(np.append(lower, i))
    hubs = np.arange(n - hub_cols, n) if hub_cols else np.zeros(0, np.int64)
    assert not own_cols or m <= n
    own = rng.permutation(n)[:m] if own_cols else None
    j_rows = []
    for r in range(m):
        k = int(rng.integers(0, row_max + 1))
        if band:
            a = int(rng.integers(0, max(1, n - band)))
            cols = a + rng.choice(min(band, n), size=min(k, band, n), replace=False)
        else:
            cols = rng.choice(n, size=min(n, k), replace=False)
        if hub_cols:
            cols = np.concatenate([cols, hubs[rng.random(hub_cols) < hub_frac]])
        if own_cols:
            cols = np.append(cols, own[r])
        j_rows.append(np.unique(cols))
    wr, wc = _csr_from_rows(w_rows, n)
    jr, jc = _csr_from_rows(j_rows, n)
    return Pattern(n, m, wr, wc, jr, jc, dict(kind="general", density=density, hub_cols=hub_cols))


def general_values(pat: Pattern, rng: np.random.Generator, sigma_lo: float, sigma_hi: float) -> Values:
    """W's off-diagonal entries ~ N(0,1) and each diagonal entry one more than
    its row's absolute off-diagonal sum over both triangles (so W is
    symmetric positive definite with eigenvalues >= 1); J ~ N(0,1); then Σx,
    Σs, b, f, g."""
    rows = np.repeat(np.arange(pat.n), np.diff(pat.w_rowptr))
    cols = pat.w_colind
    off = rows != cols
    w_vals = np.zeros(pat.nnz_w)
    w_vals[off] = rng.standard_normal(int(off.sum()))
    absum = np.zeros(pat.n)
    np.add.at(absum, rows[off], np.abs(w_vals[off]))
    np.add.at(absum, cols[off], np.abs(w_vals[off]))
    w_vals[~off] = absum[rows[~off]] + 1.0
    j_vals = rng.standard_normal(pat.nnz_j)
    return Values(w_vals, j_vals,
                  log_uniform(rng, sigma_lo, sigma_hi, pat.n),
                  log_uniform(rng, sigma_lo, sigma_hi, pat.m),
                  rng.standard_normal(pat.n), rng.standard_normal(pat.n), rng.standard_normal(pat.m))


def small_config():
    """Lifted-KKT plain: N=50, nx=8, nu=1 (n=450, m=400), Σ ~ logU[1e-2, 1e2]."""
    return nmpc_pattern(50, 8, 1), (1e-2, 1e2)


def paper_config(N: int = 2000):
    """Distillation-shaped, paper scale: N=2000, s=71 (n=142,000, m=140,000), Σ ~ logU[1e-8, 1e8]."""
    return distillation_pattern(N), (1e-8, 1e8)


def hykkt_config():
    """HyKKT gated system: the small NMPC pattern with Σx ~ logU[1e-2, 1e2]."""
    return nmpc_pattern(50, 8, 1), (1e-2, 1e2)


def batch_shapes(count: int = 256, config: int = 3):
    """(N, nx, nu) per batched instance: N ~ U{20..200}, nx ~ U{16..64}, nu ~ U{1..4}."""
    out = []
    for i in range(count):
        r = rng_for(config, i, 0)
        out.append((int(r.integers(20, 201)), int(r.integers(16, 65)), int(r.integers(1, 5))))
    return out


def serving_shapes(count: int = 16, config: int = 4, n_lo: float = 1e3, n_hi: float = 2e5):
    """Resident serving patterns: n_p ~ logU[n_lo, n_hi], nx ~ U{16..64}, nu ~ U{1..4}."""
    out = []
    for p in range(count):
        r = rng_for(config, p, 0)
        n_p = float(log_uniform(r, n_lo, n_hi, 1)[0])
        nx = int(r.integers(16, 65))
        nu = int(r.integers(1, 5))
        out.append((max(2, int(round(n_p / (nx + nu)))), nx, nu))
    return out


def poisson_arrivals(rate: float, count: int, npatterns: int, config: int = 4, stream: int = 1 << 20):
    """Arrival times (s) of a Poisson stream and the pattern id of each request."""
    r = rng_for(config, stream, 0)
    gaps = r.exponential(1.0 / rate, count)
    return np.cumsum(gaps), r.integers(0, npatterns, count)


def workload(name: str, instance: int = 0, value_set: int = 0):
    """(pattern, values) for a named workload: 'small', 'paper', 'hykkt', 'batch', 'serve'."""
    if name == "small":
        pat, (lo, hi) = small_config()
        return pat, nmpc_values(pat, rng_for(0, instance, value_set), lo, hi)
    if name == "paper":
        pat, (lo, hi) = paper_config()
        return pat, distillation_values(pat, rng_for(1, instance, value_set), lo, hi)
    if name == "hykkt":
        pat, (lo, hi) = hykkt_config()
        return pat, nmpc_values(pat, rng_for(2, instance, value_set), lo, hi)
    if name == "batch":
        N, nx, nu = batch_shapes()[instance]
        pat = nmpc_pattern(N, nx, nu)
        return pat, nmpc_values(pat, rng_for(3, instance, 1 + value_set), 1e-6, 1e6)
    if name == "serve":
        N, nx, nu = serving_shapes()[instance]
        pat = nmpc_pattern(N, nx, nu)
        return pat, nmpc_values(pat, rng_for(4, instance, 1 + value_set), 1e-6, 1e6)
    raise ValueError(name)
