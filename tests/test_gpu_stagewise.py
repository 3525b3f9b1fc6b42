"""GPU parity of the stage-structured solver (block cyclic reduction).

The condensed matrix of a dynamic program is block tridiagonal over its
stages (section "Future Works": a block-structured solver in place of the
general sparse one). Gates, as for the supernodal path: every instance's
backward error eta <= 1e-10 (recomputed here from the oracle's K); x
against the oracle's x* (condensed sparse LDL^T with refinement): with
Sigma ~ logU[1e-2, 1e2] forward error <= 1e-8 entry by entry, with the
batched workload's Sigma ~ logU[1e-6, 1e6] forward error <= 1e-13 cond_2(K);
at the paper's scale (distillation shape, N = 2000) eta <= 1e-10 and forward
error <= 1e-3 as for the supernodal path. Also: stage widths that differ
(stages merged in pairs), one- two- and three-stage horizons, repeated
refactors bitwise equal, a factor failure reported for its instance only.
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


def concat(vals, field):
    return dev(np.concatenate([getattr(v, field) for v in vals]))


def stages(pat):
    s = pat.meta["stage"]
    return np.arange(0, pat.n + 1, s, dtype=np.int32)


def solve_all(kkt, pats, vals, sps, tol=1e-14):
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    W = kkt.Stagewise(syms, sps)
    W.refactor(concat(vals, "w_vals"), concat(vals, "j_vals"), concat(vals, "sigma_x"), concat(vals, "sigma_s"))
    st, bad = W.status()
    assert (st == 0).all(), (st, bad)
    n = sum(p.n for p in pats)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    infos = W.solve(concat(vals, "b"), x, tol=tol)
    return W, x.cpu().numpy(), infos


def check_instances(pats, vals, xb, infos, wide):
    o = 0
    for q, (pat, v) in enumerate(zip(pats, vals)):
        xq = xb[o:o + pat.n]
        o += pat.n
        K = D.condensed(pat, v, v.sigma_s)
        be = D.backward_errors(K, xq, v.b)
        assert be["eta"] <= 1e-10 and infos[q]["eta"] <= 1e-10, (q, be, infos[q])
        xo, oinfo = S.lifted_solve(pat, v, v.b)
        assert oinfo["spd"]
        if wide:
            checks.assert_cond_bounded(xq, xo, K, q)
        else:
            checks.assert_well_conditioned(xq, xo, q)


@pytest.mark.parametrize("sigma", [(1e-6, 1e6), (1e-2, 1e2)], ids=["wide", "narrow"])
def test_stagewise_batch_matches_oracle(kkt, sigma):
    count = 12
    pats, vals = [], []
    for q in range(count):
        N, nx, nu = kktgen.batch_shapes()[q]
        pat = kktgen.nmpc_pattern(max(2, N // 4), nx, nu)
        pats.append(pat)
        vals.append(kktgen.nmpc_values(pat, kktgen.rng_for(3, q, 1), *sigma))
    print(f"stagewise batch of {count}, sigma {sigma}", flush=True)
    _, xb, infos = solve_all(kkt, pats, vals, [stages(p) for p in pats])
    check_instances(pats, vals, xb, infos, sigma[1] > 1e2)


@pytest.mark.parametrize("N", [1, 2, 3, 7, 50])
def test_stagewise_small_horizons(kkt, N):
    """The small NMPC shape (nx = 8, nu = 1) at horizons whose cyclic
    reduction has one, two, three, four and seven levels."""
    pat = kktgen.nmpc_pattern(N, 8, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, N, 0), 1e-2, 1e2)
    print(f"stagewise N={N}", flush=True)
    _, xb, infos = solve_all(kkt, [pat], [v], [stages(pat)])
    check_instances([pat], [v], xb, infos, False)


def test_stagewise_uneven_stages(kkt):
    """Stages merged in pairs where the index is a multiple of 3 (widths s
    and 2 s alternate irregularly): still block tridiagonal."""
    pat = kktgen.nmpc_pattern(40, 20, 3)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 77, 0), 1e-2, 1e2)
    s = pat.meta["stage"]
    sp, k = [0], 0
    while k < 40:
        k += 2 if k % 3 == 0 and k + 2 <= 40 else 1
        sp.append(k * s)
    sp = np.array(sp, dtype=np.int32)
    assert len(set(np.diff(sp))) == 2
    print(f"stagewise uneven: {len(sp) - 1} stages", flush=True)
    _, xb, infos = solve_all(kkt, [pat], [v], [sp])
    check_instances([pat], [v], xb, infos, False)


def test_stagewise_paper_scale(kkt):
    """Distillation shape, N = 2000 stages of 71 (n = 142,000), Sigma ~
    logU[1e-8, 1e8]: eta <= 1e-10, forward error <= 1e-3 against the
    oracle, for two value sets; a second refactor of the same values gives
    the same bits."""
    pat, _ = kktgen.paper_config()
    syms = [kkt.Symbolic.from_pattern(pat)]
    W = kkt.Stagewise(syms, [stages(pat)])
    for vs in (0, 1):
        _, v = kktgen.workload("paper", value_set=vs)
        print(f"stagewise paper scale value set {vs}", flush=True)
        xs = []
        for rep in range(2):
            W.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
            st, _ = W.status()
            assert st[0] == 0
            x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
            info = W.solve(dev(v.b), x)[0]
            xs.append(x.cpu().numpy())
        assert np.array_equal(xs[0], xs[1])
        K = D.condensed(pat, v, v.sigma_s)
        be = D.backward_errors(K, xs[0], v.b)
        print(vs, info, be, flush=True)
        assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
        xo, oinfo = S.lifted_solve(pat, v, v.b)
        assert oinfo["spd"]
        assert D.forward_error(xs[0], xo) <= 1e-3


def test_stagewise_failure_isolated(kkt):
    count = 5
    pats, vals = [], []
    for q in range(count):
        N, nx, nu = kktgen.batch_shapes()[q]
        pat = kktgen.nmpc_pattern(max(4, N // 8), nx, nu)
        pats.append(pat)
        vals.append(kktgen.nmpc_values(pat, kktgen.rng_for(3, q, 1), 1e-6, 1e6))
    bad_q = 2
    s = pats[bad_q].meta["stage"]
    vals[bad_q].sigma_x[2 * s:3 * s] = -1e7
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    W = kkt.Stagewise(syms, [stages(p) for p in pats])
    W.refactor(concat(vals, "w_vals"), concat(vals, "j_vals"), concat(vals, "sigma_x"), concat(vals, "sigma_s"))
    st, bad = W.status()
    print("stagewise failure", st, bad, flush=True)
    assert st[bad_q] == 4 and all(st[q] == 0 for q in range(count) if q != bad_q)
    assert 0 <= bad[bad_q] < pats[bad_q].n
    x = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError):
        W.solve(concat(vals, "b"), x)


def test_stagewise_state_and_timing(kkt):
    """A solve before any refactor is refused (STATE); per-launch timers
    count one factor launch per level and width class, and the timed solve
    equals the untimed one bit for bit."""
    pat = kktgen.nmpc_pattern(9, 8, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 9, 0), 1e-2, 1e2)
    W = kkt.Stagewise([kkt.Symbolic.from_pattern(pat)], [stages(pat)])
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError) as e:
        W.solve(dev(v.b), x)
    assert e.value.status == 3
    xs = []
    for timed in (False, True):
        W.set_timing(timed)
        W.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        W.solve(dev(v.b), x)
        xs.append(x.cpu().numpy())
    t = W.read_timing()
    print("stagewise timing", t, flush=True)
    assert t["factor"]["launches"] == 5          # 9 stages: 5 levels, one width class
    assert t["fwd"]["launches"] >= 5 and t["bwd"]["launches"] >= 5
    assert np.array_equal(xs[0], xs[1])
