"""Unstructured sparsity patterns through the HIP path, against the oracle
(run on an MI355X).

The Newton-step solves of sections "Solution 1: Lifted-KKT" and "Solution 2:
HyKKT" apply to any sparsity of W and J; these patterns have no stage
structure. W: a random lower pattern with its diagonal and diagonally
dominant values (eigenvalues >= 1); J: random rows of up to 5 columns (some
empty), and in the larger cases columns shared by about half the rows
(entries of J^T Sigma_s J with long product lists, assembled 16 lanes per
entry); Sigma ~ logU[1e-2, 1e2]. Such patterns fill in heavily (n = 1,500:
nnz(L) about 0.69 M, fronts of up to 979 rows), so they reach supernode
shapes the NMPC generators never produce; a 16 KiB LDS budget sends the
tall fronts through the HBM path. Also here: HyKKT with a full-row-rank J,
the served form, the queue schedule and the per-level launch shapes on these
trees, a band-limited pattern at n = 20,000 (also through the
stage-structured solver), and the widest supernodes allowed (128 columns).
Tolerances as in test_gpu_parity: eta <= 1e-10 against the oracle's K;
forward error and entrywise error (|x - x*| <= 1e-8 |x*| + 1e-12 ||x*||_inf)
<= 1e-8 against the oracle's solution; batched, served, queue-schedule and
launch-shape variants equal to the plain level-schedule solve bit for bit.
"""
import numpy as np
import pytest

import checks
import kktgen
from oracle import dense as D
from oracle import sparse as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (n, m, W density, shared J columns)
CASES = [(1, 0, 0.0, 0), (7, 3, 0.5, 0), (40, 30, 0.1, 0), (300, 200, 0.02, 2), (1500, 1200, 0.003, 3)]
OPTS = [dict(ordering=1), dict(ordering=2, nd_leaf=64), dict(ordering=1, front_lds_max=16 * 1024)]


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


def case(ci):
    n, m, dens, hubs = CASES[ci]
    pat = kktgen.general_pattern(kktgen.rng_for(5, ci, 0), n, m, dens, hub_cols=hubs)
    return pat, kktgen.general_values(pat, kktgen.rng_for(5, ci, 1), 1e-2, 1e2)


def plain(kkt, sym, pat, v):
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    st, bad = f.status()
    assert st == 0, bad
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    info = f.solve(dev(v.b), x)
    f.close()
    return host(x), info


@pytest.mark.parametrize("opts", OPTS, ids=["natural", "nd64", "lds16k"])
@pytest.mark.parametrize("ci", range(len(CASES)), ids=[f"n{c[0]}" for c in CASES])
def test_general_pattern_lifted(kkt, ci, opts):
    pat, v = case(ci)
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    st_ = sym.stats()
    print(f"general n={pat.n} m={pat.m} {opts}: {st_['nsuper']} fronts, {st_['levels']} levels, "
          f"up to {st_['max_rows']} rows, {st_['large_fronts']} large", flush=True)
    if "front_lds_max" in opts and ci >= 3:
        assert st_["large_fronts"] > 0
    x, info = plain(kkt, sym, pat, v)
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, x, v.b)
    assert info["eta"] <= 1e-10 and be["eta"] <= 1e-10, (info, be)
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    checks.assert_well_conditioned(x, xo)


def test_general_patterns_batched_bitwise(kkt):
    """All cases in one batch (each with its own analysis) give their plain
    solutions bit for bit."""
    pats, vals = zip(*(case(ci) for ci in range(len(CASES))))
    syms = [kkt.Symbolic.from_pattern(p, ordering=2, nd_leaf=64) for p in pats]
    xs = [plain(kkt, s, p, v)[0] for s, p, v in zip(syms, pats, vals)]
    B = kkt.Batch(syms)
    cat = lambda f: dev(np.concatenate([getattr(v, f) for v in vals]))
    B.refactor(cat("w_vals"), cat("j_vals"), cat("sigma_x"), cat("sigma_s"))
    xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    infos = B.solve(cat("b"), xb)
    assert all(i["eta"] <= 1e-10 for i in infos)
    xbh = host(xb)
    ofs = np.concatenate([[0], np.cumsum([p.n for p in pats])])
    for q in range(len(pats)):
        assert np.array_equal(xbh[ofs[q]:ofs[q + 1]], xs[q]), q
    B.close()


# HyKKT needs J of full row rank: every row also holds a column of its own
HYK_CASES = [(7, 3, 0.5, 0), (40, 30, 0.1, 0), (300, 200, 0.02, 2), (1500, 1200, 0.003, 3)]


@pytest.mark.parametrize("gamma", [1e4, 1e7])
@pytest.mark.parametrize("ci", range(len(HYK_CASES)), ids=[f"n{c[0]}" for c in HYK_CASES])
def test_general_pattern_hykkt(kkt, ci, gamma):
    """HyKKT (section "Solution 2: HyKKT") on unstructured patterns: dx and dy
    within 1e-8 of the saddle-point LDL^T, eta of the 2x2 system <= 1e-10 (the
    library's own eta within a factor 2 of the oracle's evaluation), CG
    iterations within one of the oracle's CG on the same K_gamma."""
    n, m, dens, hubs = HYK_CASES[ci]
    pat = kktgen.general_pattern(kktgen.rng_for(6, ci, 0), n, m, dens, hub_cols=hubs, own_cols=True)
    v = kktgen.general_values(pat, kktgen.rng_for(6, ci, 1), 1e-2, 1e2)
    print(f"general hykkt n={n} m={m} gamma={gamma}", flush=True)
    dx0, dy0, inn, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and inn == (pat.n, 0, pat.m)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, gamma)
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=300)
    assert info["status"] == 0, info
    dxh, dyh = host(dx), host(dy)
    assert D.forward_error(dxh, dx0) <= 1e-8 and D.forward_error(dyh, dy0) <= 1e-8
    be = D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15), (info, be)
    _, _, oinfo = S.hykkt_cg_solve(pat, v, v.f, v.g, gamma, tol=1e-10, maxit=300)
    assert abs(info["iters"] - oinfo["iters"]) <= 1, (info["iters"], oinfo["iters"])
    f.close()


def test_general_patterns_served(kkt):
    """The served form over the unstructured patterns (several requests per
    pattern, waves of up to 4 on 2 workers): each result equals the plain
    solve of its request bit for bit."""
    pats, vals = zip(*(case(ci) for ci in range(len(CASES))))
    syms = [kkt.Symbolic.from_pattern(p, ordering=2, nd_leaf=64) for p in pats]
    xs = [plain(kkt, s, p, v)[0] for s, p, v in zip(syms, pats, vals)]
    srv = kkt.Server(hbm_budget=1 << 30, max_wave=4, workers=2)
    pid = [srv.register(s) for s in syms]
    order = [q for _ in range(3) for q in range(len(pats))]
    # the server reads the request's arrays asynchronously: they stay alive until wait
    held, outs, tickets = [], [], []
    for q in order:
        v = vals[q]
        held.append([dev(getattr(v, k)) for k in ("w_vals", "j_vals", "sigma_x", "sigma_s", "b")])
        outs.append(torch.zeros(pats[q].n, dtype=torch.float64, device="cuda"))
        tickets.append(srv.submit(pid[q], *held[-1], outs[-1]))
    res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 and r["eta"] <= 1e-10 for r in res), res
    for k, q in enumerate(order):
        assert np.array_equal(host(outs[k]), xs[q]), (k, q)
    srv.close()


def test_general_patterns_queue_schedule_bitwise(kkt):
    """The persistent queue schedule on the unstructured trees (up to 67
    levels, fronts of up to 979 rows) gives the level schedule's solutions
    bit for bit, one factor per pattern and all patterns in one batch."""
    pats, vals = zip(*(case(ci) for ci in range(len(CASES))))
    syms = [kkt.Symbolic.from_pattern(p, ordering=2, nd_leaf=64) for p in pats]
    xs = []
    for s, p, v in zip(syms, pats, vals):
        f = kkt.Factor(s)
        out = []
        for sched in (kkt.SCHEDULE_LEVELS, kkt.SCHEDULE_QUEUE):
            f.set_schedule(sched)
            f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
            assert f.status()[0] == 0
            x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            assert f.solve(dev(v.b), x)["eta"] <= 1e-10
            out.append(host(x))
        assert np.array_equal(out[0], out[1]), p.n
        xs.append(out[0])
        f.close()
    B = kkt.Batch(syms)
    B.set_schedule(kkt.SCHEDULE_QUEUE)
    cat = lambda k: dev(np.concatenate([getattr(v, k) for v in vals]))
    B.refactor(cat("w_vals"), cat("j_vals"), cat("sigma_x"), cat("sigma_s"))
    xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    assert all(i["eta"] <= 1e-10 for i in B.solve(cat("b"), xb))
    xbh = host(xb)
    ofs = np.concatenate([[0], np.cumsum([p.n for p in pats])])
    for q in range(len(pats)):
        assert np.array_equal(xbh[ofs[q]:ofs[q + 1]], xs[q]), q
    B.close()


@pytest.mark.parametrize("opts", OPTS[1:], ids=["nd64", "lds16k"])
def test_general_patterns_launch_shapes_bitwise(kkt, opts):
    """The per-level launch shapes (four- or eight-wave front kernel, update
    matrices in the front's workgroup or by tiles) give the same bits on the
    unstructured trees, whose fronts (up to about 1,000 rows) are far taller
    than the four-wave kernel's fused panel path (208 rows)."""
    for ci in (3, 4):
        pat, v = case(ci)
        sym = kkt.Symbolic.from_pattern(pat, **opts)
        xs = []
        for small, split in ((0, (140, 64)), (1 << 20, (140, 64)), (1 << 20, (0, 0)), (0, (1 << 30, 0))):
            f = kkt.Factor(sym)
            f.set_small_fronts(small)
            f.set_update_split(*split)
            f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
            assert f.status()[0] == 0
            x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
            assert f.solve(dev(v.b), x)["eta"] <= 1e-10, (small, split)
            xs.append(host(x))
            f.close()
        for k in range(1, len(xs)):
            assert np.array_equal(xs[0], xs[k]), (pat.n, k)


@pytest.mark.parametrize("opts", [dict(ordering=1), dict(ordering=2, nd_leaf=200), dict(ordering=0)],
                         ids=["natural", "nd200", "auto"])
def test_banded_pattern_at_scale(kkt, opts):
    """A band-limited unstructured pattern (n = 20,000, m = 16,000, entries
    within 40 of the diagonal, as on a one-dimensional mesh): the natural
    order gives a chain of about 255 fronts, nested dissection a tree of
    about 11 levels; both solve to eta <= 1e-10 and the oracle's solution
    within 1e-8."""
    pat = kktgen.general_pattern(kktgen.rng_for(8, 0, 0), 20000, 16000, 0.3, row_max=6, band=40)
    v = kktgen.general_values(pat, kktgen.rng_for(8, 0, 1), 1e-2, 1e2)
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    st_ = sym.stats()
    print(f"banded n=20000 {opts}: {st_['nsuper']} fronts, {st_['levels']} levels", flush=True)
    x, info = plain(kkt, sym, pat, v)
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, x, v.b)
    assert info["eta"] <= 1e-10 and be["eta"] <= 1e-10, (info, be)
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    checks.assert_well_conditioned(x, xo)


def test_banded_pattern_stagewise(kkt):
    """The band-limited pattern is block tridiagonal over stages of 48
    variables (no entry couples variables more than 40 apart), so the
    stage-structured solver takes it: 417 stages, eta <= 1e-10 and the
    oracle's solution within 1e-8."""
    pat = kktgen.general_pattern(kktgen.rng_for(8, 0, 0), 20000, 16000, 0.3, row_max=6, band=40)
    v = kktgen.general_values(pat, kktgen.rng_for(8, 0, 1), 1e-2, 1e2)
    sp = np.append(np.arange(0, pat.n, 48), pat.n).astype(np.int32)
    W = kkt.Stagewise([kkt.Symbolic.from_pattern(pat)], [sp])
    W.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    st, bad = W.status()
    assert (st == 0).all(), (st, bad)
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    info = W.solve(dev(v.b), x)[0]
    xh = host(x)
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, xh, v.b)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10, (info, be)
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    checks.assert_well_conditioned(xh, xo)


WIDE = [(128, 0), (128, 64), (129, 64), (150, 60), (200, 100)]


def test_widest_supernodes(kkt):
    """The widest supernode the library allows (128 columns, max_super = 128):
    dense W blocks give fronts of 128 columns and 128-150 rows (up to 155 KB
    of LDS), the widest triangle of the sweeps' one-wave solve (two rows per
    lane) and 32 matrix-core steps per update tile; each against the oracle,
    and a batch of all of them bitwise equal to the plain solves."""
    pats, vals, syms, xs = [], [], [], []
    for n, m in WIDE:
        pat = kktgen.general_pattern(kktgen.rng_for(9, n, m), n, m, 1.0)
        v = kktgen.general_values(pat, kktgen.rng_for(9, n, m + 1), 1e-2, 1e2)
        sym = kkt.Symbolic.from_pattern(pat, ordering=1, max_super=128)
        st_ = sym.stats()
        print(f"dense n={n} m={m}: {st_['nsuper']} fronts, up to {st_['max_cols']} columns", flush=True)
        assert st_["max_cols"] == 128 or n == 200
        x, info = plain(kkt, sym, pat, v)
        K = D.condensed(pat, v, v.sigma_s)
        be = D.backward_errors(K, x, v.b)
        assert info["eta"] <= 1e-10 and be["eta"] <= 1e-10, (n, info, be)
        xo, oinfo = S.lifted_solve(pat, v, v.b)
        checks.assert_well_conditioned(x, xo, n)
        pats.append(pat), vals.append(v), syms.append(sym), xs.append(x)
    B = kkt.Batch(syms)
    cat = lambda k: dev(np.concatenate([getattr(v, k) for v in vals]))
    B.refactor(cat("w_vals"), cat("j_vals"), cat("sigma_x"), cat("sigma_s"))
    xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    assert all(i["eta"] <= 1e-10 for i in B.solve(cat("b"), xb))
    xbh = host(xb)
    ofs = np.concatenate([[0], np.cumsum([p.n for p in pats])])
    for q in range(len(pats)):
        assert np.array_equal(xbh[ofs[q]:ofs[q + 1]], xs[q]), q
    B.close()
