"""Large fronts: panels too tall for a workgroup's LDS, assembled, factored
and solved in place in HBM (run on an MI355X).

The symbolic analysis' LDS budget (kkt_options.front_lds_max) decides which
fronts are large; a small budget sends most fronts of a small system through
the HBM path, and stages 700 variables wide give fronts of about 1,460 rows,
too tall for LDS under the default budget. Tolerances as in
test_gpu_parity: eta_inf <= 1e-10 always; with Sigma in [1e-2, 1e2] the
relative forward error against the oracle <= 1e-8 and entry by entry
|x - x*| <= 1e-8 |x*| + 1e-12 ||x*||_inf; HyKKT dx and dy within 1e-8 of
the saddle-point LDL^T.
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def solve(kkt, sym, pat, v):
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    st, bad = f.status()
    assert st == 0, bad
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    info = f.solve(dev(v.b), x)
    return host(x), info, f


@pytest.mark.parametrize("budget", [8192, 16 * 1024], ids=["most-large", "mixed"])
@pytest.mark.parametrize("wide", [False, True], ids=["sigma-1e2", "sigma-1e8"])
def test_large_fronts_lifted(kkt, budget, wide):
    pat = kktgen.distillation_pattern(6)
    lo, hi = (1e-8, 1e8) if wide else (1e-2, 1e2)
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 6, 3), lo, hi)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=100, front_lds_max=budget)
    st_ = sym.stats()
    print(f"distillation N=6, LDS budget {budget}: {st_['large_fronts']} of {st_['nsuper']} fronts large", flush=True)
    assert 0 < st_["large_fronts"]
    x, info, f = solve(kkt, sym, pat, v)
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, x, v.b)
    assert info["eta"] <= 1e-10 and be["eta"] <= 1e-10, (info, be)
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    if wide:
        checks.assert_cond_bounded(x, xo, K)
    else:
        checks.assert_well_conditioned(x, xo)
    # the allocation-free solve runs the same kernels
    x2 = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f.solve_noalloc(dev(v.b), x2)
    assert np.array_equal(host(x2), x)
    # the persistent queue schedule needs every front in LDS
    with pytest.raises(kkt.KKTError):
        f.set_schedule(kkt.SCHEDULE_QUEUE)


def test_large_fronts_not_spd(kkt):
    """A negative pivot inside a large front is reported (column in the failing stage's range)."""
    pat = kktgen.distillation_pattern(6)
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 6, 4), 1e-2, 1e2)
    s = pat.meta["stage"]
    k0 = 3 * s
    v.sigma_x[k0:k0 + s] = -1e6
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=100, front_lds_max=8192)
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    st, bad = f.status()
    assert st == 4, (st, bad)
    _, oinfo = S.lifted_solve(pat, v, v.b)
    assert not oinfo["spd"]


def test_large_fronts_hykkt(kkt):
    pat = kktgen.distillation_pattern(6)
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 6, 5), 1e-2, 1e2)
    dx0, dy0, inn, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and inn == (pat.n, 0, pat.m)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=100, front_lds_max=8192)
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=200, eta_tol=1e-10)
    assert info["status"] == 0, info
    dxh, dyh = host(dx), host(dy)
    assert D.forward_error(dxh, dx0) <= 1e-8 and D.forward_error(dyh, dy0) <= 1e-8
    be = D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g)
    assert be["eta"] <= 1e-10


def test_large_fronts_batch_bitwise(kkt):
    """A batch mixing instances with and without large fronts gives each
    instance's plain solution bit for bit (no cross-instance arithmetic)."""
    pats = [kktgen.distillation_pattern(6), kktgen.distillation_pattern(5), kktgen.distillation_pattern(6)]
    vals = [kktgen.distillation_values(p, kktgen.rng_for(1, 6, 6 + q), 1e-6, 1e6) for q, p in enumerate(pats)]
    syms = [kkt.Symbolic.from_pattern(pats[0], ordering=2, nd_leaf=100, front_lds_max=8192),
            kkt.Symbolic.from_pattern(pats[1], ordering=2, nd_leaf=100),
            kkt.Symbolic.from_pattern(pats[2], ordering=2, nd_leaf=100, front_lds_max=16 * 1024)]
    xs = [solve(kkt, s, p, v)[0] for s, p, v in zip(syms, pats, vals)]
    B = kkt.Batch(syms)
    cat = lambda f: dev(np.concatenate([getattr(v, f) for v in vals]))
    B.refactor(cat("w_vals"), cat("j_vals"), cat("sigma_x"), cat("sigma_s"))
    xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    infos = B.solve(cat("b"), xb)
    assert all(i["eta"] <= 1e-10 for i in infos)
    xbh = host(xb)
    n_ofs = np.concatenate([[0], np.cumsum([p.n for p in pats])])
    for q in range(3):
        assert np.array_equal(xbh[n_ofs[q]:n_ofs[q + 1]], xs[q]), q
    with pytest.raises(kkt.KKTError):
        B.set_schedule(kkt.SCHEDULE_QUEUE)


def test_tall_fronts_default_budget(kkt):
    """Stages 700 variables wide: nested dissection gives fronts of about 1,460
    rows, too tall for LDS at any width under the default budget."""
    pat = kktgen.nmpc_pattern(4, 700, 4)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 11, 0), 1e-2, 1e2)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2)
    st_ = sym.stats()
    print(f"NMPC N=4 nx=700: {st_['large_fronts']} large fronts of {st_['nsuper']}, up to {st_['max_rows']} rows",
          flush=True)
    assert st_["large_fronts"] > 0 and st_["max_rows"] > 1300
    x, info, _ = solve(kkt, sym, pat, v)
    assert info["eta"] <= 1e-10, info
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    checks.assert_well_conditioned(x, xo)


def test_large_fronts_graph_and_served(kkt):
    """Large fronts through the batch graph (replays with new values and eager
    work between them equal the eager calls bit for bit) and through the
    served form (each result equal to the plain solve of its request)."""
    pats = [kktgen.distillation_pattern(6), kktgen.distillation_pattern(5)]
    syms = [kkt.Symbolic.from_pattern(pats[0], ordering=2, nd_leaf=100, front_lds_max=8192),
            kkt.Symbolic.from_pattern(pats[1], ordering=2, nd_leaf=100, front_lds_max=16 * 1024)]
    assert all(s.stats()["large_fronts"] > 0 for s in syms)
    sets = [[kktgen.distillation_values(p, kktgen.rng_for(1, 6, 20 + 2 * q + k), 1e-6, 1e6)
             for q, p in enumerate(pats)] for k in range(2)]
    cat = lambda vals, f: np.concatenate([getattr(v, f) for v in vals])
    B = kkt.Batch(syms)
    n = int(B.ofs["n"][-1])
    eager = []
    for vals in sets:
        B.refactor(*(dev(cat(vals, f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s")))
        x = torch.zeros(n, dtype=torch.float64, device="cuda")
        B.solve(dev(cat(vals, "b")), x)
        eager.append(host(x))
    bufs = {f: dev(cat(sets[0], f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s", "b")}
    xg = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
    B.capture(bufs["w_vals"], bufs["j_vals"], bufs["sigma_x"], bufs["sigma_s"], bufs["b"], xg, rounds=1)
    other = kkt.Factor(syms[1])
    for rep, k in enumerate((0, 1, 0)):
        for f in bufs:
            bufs[f].copy_(dev(cat(sets[k], f)))
        xg.fill_(np.nan)
        torch.cuda.synchronize()
        infos = B.replay()
        assert all(i["eta"] <= 1e-10 for i in infos)
        assert np.array_equal(host(xg), eager[k]), rep
        v1 = sets[1 - k][1]
        other.refactor(dev(v1.w_vals), dev(v1.j_vals), dev(v1.sigma_x), dev(v1.sigma_s))
        other.solve(dev(v1.b), torch.zeros(pats[1].n, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
    B.close()
    # served: each request's result equals its plain solve
    srv = kkt.Server(hbm_budget=2 << 30, max_wave=4, workers=2)
    pid = [srv.register(s) for s in syms]
    reqs = [(q % 2, k) for k in range(2) for q in range(2)] * 2
    xs, tickets, plain = [], [], []
    for p, k in reqs:
        xp, _, f = solve(kkt, syms[p], pats[p], sets[k][p])
        f.close()
        plain.append(xp)
    torch.cuda.synchronize()
    # the server reads the request's arrays asynchronously: they stay alive until wait
    held = []
    for p, k in reqs:
        v = sets[k][p]
        x = torch.zeros(pats[p].n, dtype=torch.float64, device="cuda")
        xs.append(x)
        held.append([dev(getattr(v, f)) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s", "b")])
        tickets.append(srv.submit(pid[p], *held[-1], x))
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 and r["eta"] <= 1e-10 for r in res), res
    for q in range(len(reqs)):
        assert np.array_equal(host(xs[q]), plain[q]), q
    srv.close()
