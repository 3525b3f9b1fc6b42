"""GPU checks of the two launch schedules and of the graph form.

The supernode tree can be walked one launch per level or by one persistent
launch per phase that takes fronts from a ticket counter and waits on
per-front dependency counters. Both do the same per-front arithmetic in the
same order, so the solutions must agree bitwise; the level schedule is the
one checked against the oracle elsewhere, and here each result is also
checked against the oracle's backward error (section "Hybrid linear solver":
refactor with a reused analysis, then a refined solve).

The graph form records refactor + solve once and replays it; each replay is
checked against the eager result of the same values, with eager work and
synchronisations between replays and new values written into the bound
arrays between them.
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


def plain_solve(kkt, sym, v, schedule):
    f = kkt.Factor(sym)
    f.set_schedule(schedule)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    x = torch.zeros(len(v.b), dtype=torch.float64, device="cuda")
    info = f.solve(dev(v.b), x)
    return x.cpu().numpy(), info


@pytest.mark.parametrize("case", ["nmpc-natural", "nmpc-nd", "distillation-nd"])
def test_queue_matches_levels_plain(kkt, case):
    if case.startswith("nmpc"):
        pat, (lo, hi) = kktgen.small_config()
        v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 0, 7), lo, hi)
    else:
        pat = kktgen.distillation_pattern(60)
        v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, 7), 1e-8, 1e8)
    ordering = kkt.ORDER_NATURAL if case.endswith("natural") else kkt.ORDER_ND
    print(f"{case}: n={pat.n} m={pat.m}", flush=True)
    sym = kkt.Symbolic.from_pattern(pat, ordering=ordering, nd_leaf=64 if ordering == kkt.ORDER_ND else 0)
    xl, il = plain_solve(kkt, sym, v, kkt.SCHEDULE_LEVELS)
    xq, iq = plain_solve(kkt, sym, v, kkt.SCHEDULE_QUEUE)
    assert np.array_equal(xl, xq)
    assert il["iters"] == iq["iters"] and il["eta"] == iq["eta"]
    K = D.condensed(pat, v, v.sigma_s)
    assert D.backward_errors(K, xq, v.b)["eta"] <= 1e-10
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    if case.startswith("nmpc"):
        checks.assert_well_conditioned(xq, xo)
    else:
        checks.assert_cond_bounded(xq, xo, K)


def make_batch(count, shrink, value_set=1):
    pats, vals = [], []
    for q in range(count):
        N, nx, nu = kktgen.batch_shapes()[q]
        pat = kktgen.nmpc_pattern(max(2, N // shrink), nx, nu)
        pats.append(pat)
        vals.append(kktgen.nmpc_values(pat, kktgen.rng_for(3, q, value_set), 1e-6, 1e6))
    return pats, vals


def concat(vals, field):
    return np.concatenate([getattr(v, field) for v in vals])


def check_against_oracle(pats, vals, x, n_ofs, which):
    """eta <= 1e-10 and the cond-bounded forward error against the oracle's x*
    for the instances in `which` (Sigma ~ logU[1e-6, 1e6])."""
    for q in which:
        xq = x[n_ofs[q]:n_ofs[q + 1]]
        K = D.condensed(pats[q], vals[q], vals[q].sigma_s)
        assert D.backward_errors(K, xq, vals[q].b)["eta"] <= 1e-10, q
        xo, oinfo = S.lifted_solve(pats[q], vals[q], vals[q].b)
        assert oinfo["spd"], q
        checks.assert_cond_bounded(xq, xo, K, q)


def batch_eager(B, vals, schedule):
    B.set_schedule(schedule)
    B.refactor(*[dev(concat(vals, f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s")])
    x = torch.zeros(int(B.ofs["n"][-1]), dtype=torch.float64, device="cuda")
    infos = B.solve(dev(concat(vals, "b")), x)
    return x.cpu().numpy(), infos


def test_queue_matches_levels_batch(kkt):
    count = 16
    pats, vals = make_batch(count, shrink=4)
    print(f"batch of {count}", flush=True)
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    B = kkt.Batch(syms)
    xl, il = batch_eager(B, vals, kkt.SCHEDULE_LEVELS)
    xq, iq = batch_eager(B, vals, kkt.SCHEDULE_QUEUE)
    assert np.array_equal(xl, xq)
    n_ofs = B.ofs["n"]
    for q in range(count):
        assert il[q]["iters"] == iq[q]["iters"]
    check_against_oracle(pats, vals, xq, n_ofs, range(count))


def test_queue_failure_isolated(kkt):
    count = 6
    pats, vals = make_batch(count, shrink=8)
    bad_q = 2
    s = pats[bad_q].meta["stage"]
    vals[bad_q].sigma_x[3 * s:4 * s] = -1e7
    B = kkt.Batch([kkt.Symbolic.from_pattern(p) for p in pats])
    B.set_schedule(kkt.SCHEDULE_QUEUE)
    B.refactor(*[dev(concat(vals, f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s")])
    st, bad = B.status()
    assert st[bad_q] == 4 and all(st[q] == 0 for q in range(count) if q != bad_q)
    assert bad[bad_q] >= 0


@pytest.mark.parametrize("schedule,rounds", [(0, 0), (0, 2), (1, 1)])
def test_graph_replays_match_eager(kkt, schedule, rounds):
    count = 12
    pats, vals_a = make_batch(count, shrink=4, value_set=1)
    _, vals_b = make_batch(count, shrink=4, value_set=2)
    print(f"graph: batch of {count}, schedule {schedule}, rounds {rounds}", flush=True)
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    B = kkt.Batch(syms)
    xa, ia = batch_eager(B, vals_a, schedule)
    xb, ib = batch_eager(B, vals_b, schedule)
    check_against_oracle(pats, vals_a, xa, B.ofs["n"], range(count))
    # arrays bound to the graph
    bufs = {f: dev(concat(vals_a, f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s", "b")}
    x = torch.full((int(B.ofs["n"][-1]),), np.nan, dtype=torch.float64, device="cuda")
    B.capture(bufs["w_vals"], bufs["j_vals"], bufs["sigma_x"], bufs["sigma_s"], bufs["b"], x, rounds=rounds)
    other = kkt.Factor(syms[0])
    for rep, (vals, xe, ie) in enumerate([(vals_a, xa, ia), (vals_b, xb, ib), (vals_a, xa, ia), (vals_a, xa, ia)]):
        for f in bufs:
            bufs[f].copy_(dev(concat(vals, f)))
        x.fill_(np.nan)
        torch.cuda.synchronize()
        infos = B.replay()
        got = x.cpu().numpy()
        assert np.array_equal(got, xe), rep
        assert [i["iters"] for i in infos] == [i["iters"] for i in ie], rep
        # eager work of the program between replays
        v0 = vals_b[0] if rep % 2 == 0 else vals_a[0]
        other.refactor(dev(v0.w_vals), dev(v0.j_vals), dev(v0.sigma_x), dev(v0.sigma_s))
        y = torch.zeros(pats[0].n, dtype=torch.float64, device="cuda")
        other.solve(dev(v0.b), y)
        torch.cuda.synchronize()
    # the eager calls still work on the batch after the graph replays
    xe2, _ = batch_eager(B, vals_b, schedule)
    assert np.array_equal(xe2, xb)


def test_queue_full_batch_repeated(kkt):
    """Full-size instances under the queue schedule, refactored several times:
    every instance factors (no spurious NOT_SPD) and every solution equals the
    level schedule's bitwise."""
    count = 128
    shapes = kktgen.batch_shapes(count)
    pats = [kktgen.nmpc_pattern(*sh) for sh in shapes]
    vals = [kktgen.nmpc_values(p, kktgen.rng_for(3, q, 1), 1e-6, 1e6) for q, p in enumerate(pats)]
    print(f"queue: {count} full-size instances", flush=True)
    syms = [kkt.Symbolic.from_pattern(p, ordering=kkt.ORDER_ND, nd_leaf=256, max_super=96) for p in pats]
    B = kkt.Batch(syms)
    xl, il = batch_eager(B, vals, kkt.SCHEDULE_LEVELS)
    check_against_oracle(pats, vals, xl, B.ofs["n"], range(0, count, 16))
    for rep in range(4):
        xq, iq = batch_eager(B, vals, kkt.SCHEDULE_QUEUE)
        st, bad = B.status()
        assert not st.any(), (rep, np.nonzero(st)[0].tolist())
        assert np.array_equal(xl, xq), rep
