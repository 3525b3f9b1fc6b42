"""GPU parity of the batched form (many NMPC instances per launch).

Gates: every instance's backward error eta <= 1e-10; every instance's x
against the oracle's x* (condensed sparse LDL^T with refinement): with
Sigma ~ logU[1e-2, 1e2] forward error <= 1e-8 and |x - x*| <= 1e-8 |x*| +
1e-12 ||x*||_inf entry by entry, with the batched workload's
Sigma ~ logU[1e-6, 1e6] forward error <= 1e-13 cond_2(K); each instance's
batched solution is bitwise identical to the same instance solved alone by a
plain factor (identical per-instance operation order, no cross-instance
reductions); a factor failure in one instance is reported for that instance
only. Instance shapes follow the batched workload: N ~ U{20..200},
nx ~ U{16..64}, nu ~ U{1..4}.
"""
import numpy as np
import pytest

import checks
import kktgen
from oracle import dense as D
from oracle import sparse as S

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


def make_batch(count, shrink=1, sigma=(1e-6, 1e6)):
    pats, vals = [], []
    for q in range(count):
        N, nx, nu = kktgen.batch_shapes()[q]
        N = max(2, N // shrink)
        pat = kktgen.nmpc_pattern(N, nx, nu)
        pats.append(pat)
        vals.append(kktgen.nmpc_values(pat, kktgen.rng_for(3, q, 1), *sigma))
    return pats, vals


def concat(vals, field):
    return dev(np.concatenate([getattr(v, field) for v in vals]))


@pytest.mark.parametrize("sigma", [(1e-6, 1e6), (1e-2, 1e2)], ids=["wide", "narrow"])
@pytest.mark.parametrize("ordering", [1, 2])
def test_batch_matches_oracle_and_plain(kkt, ordering, sigma):
    count = 12
    pats, vals = make_batch(count, shrink=4, sigma=sigma)
    print(f"batch of {count}, ordering {ordering}, sigma {sigma}", flush=True)
    syms = [kkt.Symbolic.from_pattern(p, ordering=ordering) for p in pats]
    B = kkt.Batch(syms)
    n_ofs = B.ofs["n"]
    B.refactor(concat(vals, "w_vals"), concat(vals, "j_vals"), concat(vals, "sigma_x"), concat(vals, "sigma_s"))
    st, bad = B.status()
    assert (st == 0).all()
    x = torch.zeros(int(n_ofs[-1]), dtype=torch.float64, device="cuda")
    infos = B.solve(concat(vals, "b"), x)
    xb = x.cpu().numpy()
    for q in range(count):
        pat, v = pats[q], vals[q]
        xq = xb[n_ofs[q]:n_ofs[q + 1]]
        K = D.condensed(pat, v, v.sigma_s)
        be = D.backward_errors(K, xq, v.b)
        assert be["eta"] <= 1e-10 and infos[q]["eta"] <= 1e-10, (q, be, infos[q])
        xo, oinfo = S.lifted_solve(pat, v, v.b)
        assert oinfo["spd"]
        if sigma[1] <= 1e2:
            checks.assert_well_conditioned(xq, xo, q)
        else:
            checks.assert_cond_bounded(xq, xo, K, q)
        # plain factor of the same instance: bitwise identical
        f = kkt.Factor(syms[q])
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        xp = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        pinfo = f.solve(dev(v.b), xp)
        assert np.array_equal(xp.cpu().numpy(), xq), q
        assert pinfo["iters"] == infos[q]["iters"]


def test_batch_failure_isolated(kkt):
    count = 6
    pats, vals = make_batch(count, shrink=8)
    bad_q = 3
    s = pats[bad_q].meta["stage"]
    vals[bad_q].sigma_x[2 * s:3 * s] = -1e7
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    B = kkt.Batch(syms)
    B.refactor(concat(vals, "w_vals"), concat(vals, "j_vals"), concat(vals, "sigma_x"), concat(vals, "sigma_s"))
    st, bad = B.status()
    assert st[bad_q] == 4 and all(st[q] == 0 for q in range(count) if q != bad_q)
    assert bad[bad_q] >= 0
    # the solve still serves the other instances: each equals its plain solve bit for bit
    x = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError) as ei:
        B.solve(concat(vals, "b"), x)
    assert ei.value.status == 4
    xb = x.cpu().numpy()
    o = 0
    for q, (p, v, sym) in enumerate(zip(pats, vals, syms)):
        if q != bad_q:
            f = kkt.Factor(sym)
            f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
            xq = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            f.solve(dev(v.b), xq)
            assert np.array_equal(xb[o:o + p.n], xq.cpu().numpy()), q
            f.close()
        o += p.n


def test_batch_shared_symbolic(kkt):
    """The same analysis reused for several instances (one upload)."""
    pat = kktgen.nmpc_pattern(30, 20, 2)
    vals = [kktgen.nmpc_values(pat, kktgen.rng_for(3, 900, vs), 1e-6, 1e6) for vs in range(5)]
    sym = kkt.Symbolic.from_pattern(pat)
    B = kkt.Batch([sym] * 5)
    B.refactor(concat(vals, "w_vals"), concat(vals, "j_vals"), concat(vals, "sigma_x"), concat(vals, "sigma_s"))
    x = torch.zeros(5 * pat.n, dtype=torch.float64, device="cuda")
    infos = B.solve(concat(vals, "b"), x)
    xb = x.cpu().numpy()
    for q in range(5):
        K = D.condensed(pat, vals[q], vals[q].sigma_s)
        assert D.backward_errors(K, xb[q * pat.n:(q + 1) * pat.n], vals[q].b)["eta"] <= 1e-10


def test_autotuned_shapes_applied(kkt):
    """The batch autotuner's pick (options, schedule, update split, four-wave
    column threshold) and the single-pattern tuner's pick are valid settings:
    applied to a batch and to a factor they give eta <= 1e-10 and the same
    bits as the library's default launch shapes on the same analyses."""
    from paper_2403_15913_amd import autotune
    pats, vals = make_batch(8, shrink=4)
    tuned = autotune.tune_batch(pats, vals, reps=1)
    best = tuned["best"]
    print("batch pick", best, flush=True)
    assert {"ordering", "nd_leaf", "max_super", "schedule", "small", "split"} <= set(best)
    assert best["small"] in autotune.SMALLS and tuple(best["split"]) in autotune.SPLITS
    syms = autotune.analyze_many(pats, **{k: best[k] for k in ("ordering", "nd_leaf", "max_super")})
    cat = [concat(vals, f) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s")]
    b = concat(vals, "b")
    xs = []
    for tuned_shapes in (True, False):
        B = kkt.Batch(syms)
        if tuned_shapes:
            B.set_schedule(best["schedule"])
            B.set_small_fronts(best["small"])
            B.set_update_split(*best["split"])
        B.refactor(*cat)
        x = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
        infos = B.solve(b, x)
        assert all(i["eta"] <= 1e-10 for i in infos)
        torch.cuda.synchronize()
        xs.append(x.cpu().numpy())
        B.close()
    assert np.array_equal(xs[0], xs[1])
    # one pattern
    pat, v = pats[0], vals[0]
    pick = autotune.tune_pattern(pat, v, reps=1, table_path=None)
    print("pattern pick", pick, flush=True)
    sym = kkt.Symbolic.from_pattern(pat, **{k: pick[k] for k in ("ordering", "nd_leaf", "max_super")})
    xp = []
    for tuned_shapes in (True, False):
        f = kkt.Factor(sym)
        if tuned_shapes:
            f.set_schedule(pick["schedule"])
            f.set_update_split(*pick["split"])
            f.set_small_fronts(pick["small"])
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        assert f.solve(dev(v.b), x)["eta"] <= 1e-10
        torch.cuda.synchronize()
        xp.append(x.cpu().numpy())
        f.close()
    assert np.array_equal(xp[0], xp[1])
