"""General HyKKT (equality rows G and inequality rows H with slack weights)
through the C ABI, against the FP64 oracle.

The factor holds K_gamma = W + Sigma_x + H^T D_s H + gamma G^T G and the
Schur-complement CG runs over the equality rows only (section "Solution 2:
HyKKT", eqs. (hykkt), (schurcomp), with the condensed matrix of eq.
(kkt:condensed)). Tolerances: dx and dy within a relative forward error of
1e-8 of Bunch-Kaufman on [[K_k, G^T], [G, 0]] (Sigma in [1e-2, 1e2]), the
saddle system's eta <= 1e-10 by the oracle's evaluator with the library's own
eta within a factor of 2, dy exactly 0 on the inequality rows, the CG count
within the classical bound for kappa(S_gamma); the slack and multiplier steps
recovered from dx match the augmented system with both row kinds to 1e-8.
"""
import numpy as np
import pytest

import kktgen
from oracle import dense as D

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def kkt():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15913_amd import kkt as K
    K.lib()
    return K


def dev(a):
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("gamma", [1e4, 1e7])
@pytest.mark.parametrize("split", ["alternate", "first_half"])
@pytest.mark.parametrize("shape", ["nmpc", "unstructured"])
def test_general_hykkt_matches_oracle(kkt, gamma, split, shape):
    if shape == "nmpc":
        pat, v = kktgen.workload("small", instance=3)
    else:
        # no stage structure; every row of J holds a column of its own (full row rank)
        pat = kktgen.general_pattern(kktgen.rng_for(99, 0, 0), 300, 200, 0.02, hub_cols=2, own_cols=True)
        v = kktgen.general_values(pat, kktgen.rng_for(99, 0, 1), 1e-2, 1e2)
    eq = np.arange(0, pat.m, 2) if split == "alternate" else np.arange(pat.m // 2)
    G, H, dsw, eqi, ineq = D.split_rows(pat, v, eq)
    n, me, mi = pat.n, len(eqi), len(ineq)
    rng = kktgen.rng_for(98, 0, int(gamma))
    r1, r2, r3, r4 = (rng.standard_normal(k) for k in (n, mi, me, mi))
    fv = -(r1 + H.T @ (dsw * r4 - r2))
    g = np.zeros(pat.m)
    g[eqi] = -r3
    print(f"general hykkt {shape} gamma={gamma} split={split}", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    f.set_equality_rows(eq)
    with pytest.raises(kkt.KKTError):
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s), 0.0)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s), gamma)
    assert f.status()[0] == 0
    dx = torch.zeros(n, dtype=torch.float64, device="cuda")
    dy = torch.full((pat.m,), float("nan"), dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(fv), dev(g), dx, dy, tol=1e-10, maxit=300)
    assert info["status"] == 0, info
    dxh, dyh = host(dx), host(dy)
    assert np.all(dyh[ineq] == 0.0)
    A = D.general_hykkt_saddle(pat, v, eq, 0.0)
    rhs = np.concatenate([fv, -r3])
    zs = D.bunch_kaufman(A).solve(rhs)
    assert D.forward_error(dxh, zs[:n]) <= 1e-8 and D.forward_error(dyh[eqi], zs[n:]) <= 1e-8
    be = D.backward_errors(A, np.concatenate([dxh, dyh[eqi]]), rhs)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15), (info, be)
    # CG count within the classical bound for the Schur complement's conditioning
    Kg = D.general_hykkt_saddle(pat, v, eq, gamma)[:n, :n]
    ev = np.linalg.eigvalsh(G @ np.linalg.solve(Kg, G.T))
    assert info["iters"] <= D.cg_iteration_bound(ev.max() / ev.min(), 1e-10) + 1, info
    # the whole augmented system with both row kinds (eq. (kkt:augmented))
    za = np.linalg.solve(D.general_augmented(pat, v, eq), -np.concatenate([r1, r2, r3, r4]))
    ds_rec = -r4 - H @ dxh
    dz_rec = -r2 - dsw * ds_rec
    assert D.forward_error(ds_rec, za[n:n + mi]) <= 1e-8 and D.forward_error(dz_rec, za[n + mi + me:]) <= 1e-8


def test_equality_rows_cleared(kkt):
    """count = 0 returns the factor to the Lifted-KKT rules (bitwise the same
    solution as a factor that never had equality rows)."""
    pat, v = kktgen.workload("small", instance=1)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    f.set_equality_rows(np.arange(10))
    f.set_equality_rows([])
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f.solve(dev(v.b), x)
    f2 = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    f2.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    x2 = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f2.solve(dev(v.b), x2)
    assert np.array_equal(host(x), host(x2))
