"""GPU tests of the served form (continuous batching over resident patterns).

Gates: every served result has eta <= 1e-10 against the oracle evaluator;
a request's result is bitwise the same served alone (waves of one) and in a
mix of many concurrent requests of different patterns (A20's design goal;
the gate is bitwise); a request that cannot fit the HBM budget is refused
with BUDGET; statistics count every request; a request whose factor fails
(NOT_SPD) fails alone, its wave's other requests unchanged bit for bit.
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


def patterns(count=4):
    out = []
    for p in range(count):
        N, nx, nu = kktgen.serving_shapes()[p]
        N = max(2, min(N, 120))
        pat = kktgen.nmpc_pattern(N, nx, nu)
        out.append(pat)
    return out


def values(pat, p, r):
    return kktgen.nmpc_values(pat, kktgen.rng_for(4, p, 1 + r), 1e-6, 1e6)


def upload(v):
    return [dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s), dev(v.b)]


def test_alone_vs_mix(kkt):
    pats = patterns(4)
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    reqs = [(q % 4, q) for q in range(24)]
    vals = [values(pats[p], p, r) for p, r in reqs]
    dvals = [upload(v) for v in vals]
    # alone: one request per wave, one worker
    alone = kkt.Server(hbm_budget=2 << 30, max_wave=1, workers=1)
    pid = [alone.register(s) for s in syms]
    xa = []
    for (p, r), dv in zip(reqs, dvals):
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        t = alone.submit(pid[p], *dv, x)
        res = alone.wait(t)
        assert res["status"] == 0, res
        xa.append(x.cpu().numpy())
    assert alone.stats()["waves"] == len(reqs)
    alone.close()
    # mix: all submitted at once, several waves in flight
    mix = kkt.Server(hbm_budget=2 << 30, max_wave=8, workers=2)
    pid = [mix.register(s) for s in syms]
    xs, tickets = [], []
    for (p, r), dv in zip(reqs, dvals):
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        xs.append(x)
        tickets.append(mix.submit(pid[p], *dv, x))
    res = [mix.wait(t) for t in tickets]
    st = mix.stats()
    assert st["completed"] == len(reqs) and st["waves"] < len(reqs) and st["p99_s"] >= st["p50_s"] > 0
    for q, ((p, r), v) in enumerate(zip(reqs, vals)):
        assert res[q]["status"] == 0
        xm = xs[q].cpu().numpy()
        assert np.array_equal(xm, xa[q]), q
        K = D.condensed(pats[p], v, v.sigma_s)
        assert D.backward_errors(K, xm, v.b)["eta"] <= 1e-10
    mix.close()


def test_budget_refusal(kkt):
    pat = patterns(1)[0]
    sym = kkt.Symbolic.from_pattern(pat)
    srv = kkt.Server(hbm_budget=1 << 20, max_wave=4, workers=1)
    with pytest.raises(kkt.KKTError) as ei:
        srv.register(sym)
    assert ei.value.status == 9
    srv.close()


def test_small_budget_forces_small_waves(kkt):
    pats = patterns(2)
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    from paper_2403_15913_amd import kkt as K
    # smallest budget that admits the larger pattern, then room for about two requests
    budget = 1 << 20
    while True:
        probe = K.Server(hbm_budget=budget, max_wave=64, workers=1)
        try:
            for s in syms:
                probe.register(s)
            break
        except K.KKTError as e:
            assert e.status == 9
            budget *= 2
        finally:
            probe.close()
    srv = K.Server(hbm_budget=int(budget * 1.5), max_wave=64, workers=1)
    pid = [srv.register(s) for s in syms]
    tickets, xs, vals, keep = [], [], [], []
    for q in range(10):
        p = q % 2
        v = values(pats[p], p, 100 + q)
        vals.append((p, v))
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        xs.append(x)
        keep.append(upload(v))  # inputs must stay alive until the request is done
        tickets.append(srv.submit(pid[p], *keep[-1], x))
    for t in tickets:
        assert srv.wait(t)["status"] == 0
    st = srv.stats()
    assert st["completed"] == 10 and st["waves"] >= 2
    for (p, v), x in zip(vals, xs):
        K = D.condensed(pats[p], v, v.sigma_s)
        assert D.backward_errors(K, x.cpu().numpy(), v.b)["eta"] <= 1e-10
    srv.close()


def test_served_failure_isolated(kkt):
    """A request whose K is not positive definite (Sigma_x strongly negative on
    some variables) fails with NOT_SPD (4) alone: the other requests of its
    waves finish with status 0 and the results they get alone, bit for bit;
    the server keeps serving afterwards."""
    pats = patterns(3)
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    bad_q = 4
    reqs = [(q % 3, q) for q in range(9)]
    vals = []
    for p, q in reqs:
        v = values(pats[p], p, 200 + q)
        if q == bad_q:
            v.sigma_x[: pats[p].n // 4] = -1e9
        vals.append(v)
    # alone: waves of one
    alone = kkt.Server(hbm_budget=2 << 30, max_wave=1, workers=1)
    pid = [alone.register(s) for s in syms]
    xa, keep = [], []
    for (p, q), v in zip(reqs, vals):
        if q == bad_q:
            xa.append(None)
            continue
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        keep.append(upload(v))
        assert alone.wait(alone.submit(pid[p], *keep[-1], x))["status"] == 0
        xa.append(x.cpu().numpy())
    alone.close()
    # mixed: one wave of all nine on one worker, the failing request among them
    mix = kkt.Server(hbm_budget=2 << 30, max_wave=16, workers=1, linger_us=20000.0)
    pid = [mix.register(s) for s in syms]
    xs, tickets, keep = [], [], []
    for (p, q), v in zip(reqs, vals):
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        xs.append(x)
        keep.append(upload(v))
        tickets.append(mix.submit(pid[p], *keep[-1], x))
    res = [mix.wait(t) for t in tickets]
    for (p, q), r, x, a in zip(reqs, res, xs, xa):
        if q == bad_q:
            assert r["status"] == 4, r
        else:
            assert r["status"] == 0, (q, r)
            assert np.array_equal(x.cpu().numpy(), a), q
    # still serving
    p, v = 0, values(pats[0], 0, 300)
    x = torch.zeros(pats[0].n, dtype=torch.float64, device="cuda")
    keep.append(upload(v))
    assert mix.wait(mix.submit(pid[p], *keep[-1], x))["status"] == 0
    K = D.condensed(pats[0], v, v.sigma_s)
    assert D.backward_errors(K, x.cpu().numpy(), v.b)["eta"] <= 1e-10
    mix.close()
