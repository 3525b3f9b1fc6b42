"""GPU parity of the HIP library against the FP64 oracle (run on an MI355X).

Tolerances (stated per test):
  * backward error eta_inf <= 1e-10 in every case (the library's gate);
  * Lifted-KKT, Sigma in [1e-2, 1e2]: relative forward error <= 1e-8 and,
    entry by entry, |x - x*| <= 1e-8 |x*| + 1e-12 ||x*||_inf (tests/checks.py);
    wider Sigma ranges: forward error <= 1e-13 cond_2(K);
  * HyKKT: dx and dy each within a relative forward error of 1e-8 of the
    saddle-point LDL^T for gamma in {1e4, 1e6, 1e7, 1e8} (normwise: the
    error HyKKT adds grows with gamma and is not small entry by entry; the
    oracle's own CG and its LDL^T differ by up to 6e-7 componentwise at
    gamma = 1e8), eta on the 2x2 system <= 1e-10, CG iteration count within
    one of the oracle's;
  * HyKKT with Sigma_x ~ logU[1e-8, 1e8] on the small system (saddle condition
    number ~1e15): eta <= 1e-10, forward error <= 1e-7 against Bunch-Kaufman,
    CG count within two of the oracle's;
  * HyKKT at paper scale: CG count within one of the oracle's for each value
    set, eta <= 1e-10, dx and dy within 1e-6 of the saddle-point LDL^T (the
    oracle's CG and LDL^T themselves differ by 8e-8 there: J is nearly
    singular, sigma_min ~ 1e-4).
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


def lifted_run(kkt, pat, v, sym=None, **kw):
    sym = sym or kkt.Symbolic.from_pattern(pat, **kw)
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    st, bad = f.status()
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    info = f.solve(dev(v.b), x) if st == 0 else None
    return st, bad, (host(x) if st == 0 else None), info, f


ORDERINGS = [dict(ordering=1), dict(ordering=2, nd_leaf=64), dict(ordering=1, max_super=1, relax_small=-1, relax_frac=0.0)]


@pytest.mark.parametrize("kw", ORDERINGS, ids=["natural", "nd64", "scalar"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_small_lifted(kkt, kw, seed):
    pat, v = kktgen.workload("small", instance=seed)
    print(f"small lifted seed={seed} {kw}", flush=True)
    st, bad, x, info, _ = lifted_run(kkt, pat, v, **kw)
    assert st == 0, bad
    xs, inn = D.lifted_solution(pat, v, v.b)
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, x, v.b)
    assert info["eta"] <= 1e-10 and be["eta"] <= 1e-10
    # at eta ~ 1e-17 both values are rounding noise of the residual itself
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15)
    checks.assert_well_conditioned(x, xs)


def test_small_ill_conditioned(kkt):
    pat, _ = kktgen.small_config()
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 7, 0), 1e-8, 1e8)
    st, bad, x, info, _ = lifted_run(kkt, pat, v, ordering=2, nd_leaf=64)
    assert st == 0
    K = D.condensed(pat, v, v.sigma_s)
    be = D.backward_errors(K, x, v.b)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
    xo, _ = S.lifted_solve(pat, v, v.b)
    checks.assert_cond_bounded(x, xo, K)


def test_not_spd_detected(kkt):
    pat, v = kktgen.workload("small", instance=2)
    s = pat.meta["stage"]
    k0 = 20 * s
    v.sigma_x[k0:k0 + s] = -1e4
    st, bad, x, info, f = lifted_run(kkt, pat, v, ordering=2, nd_leaf=64)
    assert st == 4 and k0 - s <= bad < k0 + 2 * s
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert not oinfo["spd"]
    # a solve on the failed factor is refused
    with pytest.raises(kkt.KKTError):
        f.solve(dev(v.b), torch.zeros(pat.n, dtype=torch.float64, device="cuda"))


def test_nonfinite_detected(kkt):
    pat, v = kktgen.workload("small", instance=3)
    v.w_vals[17] = np.nan
    st, bad, x, info, _ = lifted_run(kkt, pat, v, ordering=1)
    assert st == 5


def test_repeat_bitwise(kkt):
    pat, v = kktgen.workload("small", instance=4)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64)
    _, _, x1, _, _ = lifted_run(kkt, pat, v, sym=sym)
    _, _, x2, _, _ = lifted_run(kkt, pat, v, sym=sym)
    assert np.array_equal(x1, x2)


def test_refactor_new_values_same_factor(kkt):
    pat, v0 = kktgen.workload("small", instance=5)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64)
    f = kkt.Factor(sym)
    for vs in range(3):
        _, v = kktgen.workload("small", instance=5, value_set=vs)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info = f.solve(dev(v.b), x)
        xs, _ = D.lifted_solution(pat, v, v.b)
        assert info["eta"] <= 1e-10
        checks.assert_well_conditioned(host(x), xs, vs)


def test_matvec(kkt):
    pat, v = kktgen.workload("small", instance=6)
    _, _, _, _, f = lifted_run(kkt, pat, v, ordering=1)
    xv = np.random.default_rng(0).standard_normal(pat.n)
    y = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f.matvec(dev(xv), y)
    K = D.condensed(pat, v, v.sigma_s)
    ref = K @ xv
    assert np.abs(host(y) - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("mode", ["lifted", "hykkt"])
def test_matvec_long_product_lists(kkt, mode):
    """K x on the distillation pattern, whose per-stage coupling columns give
    entries of K with up to 70 products of J entries (assembled 16 lanes per
    entry): Lifted-KKT K = W + Sigma_x + J^T Sigma_s J (eq. (liftedkkt)) and
    K_gamma = W + Sigma_x + gamma J^T J (eq. (hykkt)) against the oracle's
    explicit matrix, to 1e-13 of the largest entry of the product."""
    pat = kktgen.distillation_pattern(8)
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, 11), 1e-2, 1e2)
    print(f"matvec {mode}: n={pat.n} m={pat.m}", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    if mode == "lifted":
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        K = D.condensed(pat, v, v.sigma_s)
    else:
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e4)
        K = D.condensed(pat, v, np.full(pat.m, 1e4))
    assert f.status()[0] == 0
    xv = np.random.default_rng(5).standard_normal(pat.n)
    y = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f.matvec(dev(xv), y)
    ref = K @ xv
    assert np.abs(host(y) - ref).max() <= 1e-13 * np.abs(ref).max()


def test_edge_no_constraints_and_single_stage(kkt):
    # m = 0: K = W + Sigma_x
    pat = kktgen.nmpc_pattern(7, 3, 2)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(93, 0, 0), 1e-2, 1e2)
    empty = kktgen.Pattern(pat.n, 0, pat.w_rowptr, pat.w_colind, np.zeros(1, np.int32), np.zeros(0, np.int32), pat.meta)
    ve = kktgen.Values(v.w_vals, np.zeros(0), v.sigma_x, np.zeros(0), v.b, v.f, np.zeros(0))
    st, bad, x, info, _ = lifted_run(kkt, empty, ve, ordering=1)
    K = D.condensed(empty, ve, ve.sigma_s).toarray()
    assert st == 0 and D.forward_error(x, np.linalg.solve(K, ve.b)) <= 1e-12
    # N = 1: one dense front
    pat = kktgen.nmpc_pattern(1, 5, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(93, 1, 0), 1e-2, 1e2)
    st, bad, x, info, _ = lifted_run(kkt, pat, v)
    K = D.condensed(pat, v, v.sigma_s).toarray()
    assert st == 0 and D.forward_error(x, np.linalg.solve(K, v.b)) <= 1e-12


@pytest.mark.parametrize("gamma", [1e4, 1e6, 1e7, 1e8])
def test_hykkt_gamma(kkt, gamma):
    pat, v = kktgen.workload("hykkt")
    print(f"hykkt gamma={gamma}", flush=True)
    dx0, dy0, inn, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and inn == (pat.n, 0, pat.m)
    sym = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64)
    f = kkt.Factor(sym)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, gamma)
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=200)
    assert info["status"] == 0
    dxh, dyh = host(dx), host(dy)
    assert D.forward_error(dxh, dx0) <= 1e-8 and D.forward_error(dyh, dy0) <= 1e-8
    be = D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g)
    assert be["eta"] <= 1e-10
    check_device_eta(info, be)
    _, _, oinfo = S.hykkt_cg_solve(pat, v, v.f, v.g, gamma, tol=1e-10)
    assert abs(info["iters"] - oinfo["iters"]) <= 1


def check_device_eta(info, be):
    """The library's eta of the saddle system (its own residual kernels)
    against the oracle's evaluation of the same (dx, dy): both are rounding
    noise of the same residual, so they agree within a factor of 2 or 1e-15."""
    assert info["eta"] <= 1e-10
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15), (info, be)


def test_solve_async_matches_sync(kkt):
    """kkt_solve without an info record is asynchronous (stop decisions on
    the device, the rounds after the stop do nothing): the same x bit for bit
    as the host-driven solve, for a solve that refines and one that stops at
    once (max_iter = 0)."""
    pat, v = kktgen.workload("small", instance=5)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 5, 3), 1e-8, 1e8)
    print("solve async vs sync", flush=True)
    st, bad, x_sync, info, f = lifted_run(kkt, pat, v, ordering=2, nd_leaf=64)
    assert st == 0
    # tol = 0: refinement runs until omega stops halving or max_iter
    for max_iter, tol in ((10, 0.0), (10, 1e-14), (0, 0.0)):
        xs = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        si = f.solve(dev(v.b), xs, max_iter=max_iter, tol=tol)
        assert si["iters"] >= (1 if max_iter and tol == 0.0 else 0), si
        xa = torch.full((pat.n,), float("nan"), dtype=torch.float64, device="cuda")
        assert f.solve(dev(v.b), xa, max_iter=max_iter, tol=tol, info=False) is None
        assert f.status()[0] == 0
        assert np.array_equal(host(xa), host(xs)), (max_iter, tol)


def test_cg_async_matches_sync(kkt):
    """kkt_cg_schur without an info record queues maxit iterations whose
    stop decisions are taken on the device: dx and dy equal the synchronous
    call's bit for bit (recurrence stop and eta stop)."""
    pat, v = kktgen.workload("hykkt")
    print("cg async vs sync", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e4)
    for eta_tol in (0.0, 1e-12):
        out = []
        for info in (True, False):
            dx = torch.full((pat.n,), float("nan"), dtype=torch.float64, device="cuda")
            dy = torch.full((pat.m,), float("nan"), dtype=torch.float64, device="cuda")
            ci = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=40, eta_tol=eta_tol, info=info)
            if info:
                assert ci["status"] == 0 and ci["iters"] < 40, ci
            out.append((host(dx), host(dy)))
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1]), eta_tol


def test_cg_on_lifted_factor_refused(kkt):
    pat, v = kktgen.workload("small", instance=7)
    _, _, _, _, f = lifted_run(kkt, pat, v, ordering=1)
    z = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    zm = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError):
        f.cg_schur(z, zm, z.clone(), zm.clone())


@pytest.mark.parametrize("opts", [{}, dict(ordering=2, nd_leaf=417, max_super=96)], ids=["default", "bench"])
def test_paper_scale_lifted(kkt, opts):
    """Distillation shape, N=2000 (n=142,000): eta <= 1e-10 for two value sets,
    with the default symbolic options and with the options bench.py's
    autotuner picks for this pattern (the timed configuration)."""
    pat, v = kktgen.workload("paper")
    print(f"paper-scale lifted {opts}", flush=True)
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    f = kkt.Factor(sym)
    for vs in (0, 1):
        if vs:
            _, v = kktgen.workload("paper", value_set=vs)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        assert f.status()[0] == 0
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info = f.solve(dev(v.b), x)
        xh = host(x)
        K = D.condensed(pat, v, v.sigma_s)
        be = D.backward_errors(K, xh, v.b)
        print(vs, info, be, flush=True)
        assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
        xo, oinfo = S.lifted_solve(pat, v, v.b)
        assert oinfo["spd"]
        # both solutions are backward stable; their difference is bounded by
        # the conditioning (forward error is reported, gated loosely)
        assert D.forward_error(xh, xo) <= 1e-3


@pytest.mark.parametrize("shape,opts", [((4, 300, 4), dict(ordering=1)), ((8, 120, 6), dict(ordering=2, nd_leaf=64))],
                         ids=["natural-353rows", "nd-313rows"])
def test_tall_fronts(kkt, shape, opts):
    """Fronts taller than the fused panel path covers (more than 272 rows:
    the pivot chain by one wave and a separate triangular solve): eta <=
    1e-10, forward error <= 1e-8 against the oracle (Sigma in [1e-2, 1e2]),
    and the queue schedule bitwise equal to the level schedule."""
    pat = kktgen.nmpc_pattern(*shape)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(95, 0, 0), 1e-2, 1e2)
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    cp, _, nr = sym.supernodes()
    print(f"tall fronts {shape} {opts}: max rows {max(nr)}", flush=True)
    assert max(nr) > 272
    xs = []
    for sched in (kkt.SCHEDULE_LEVELS, kkt.SCHEDULE_QUEUE):
        f = kkt.Factor(sym)
        f.set_schedule(sched)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        assert f.status()[0] == 0
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info = f.solve(dev(v.b), x)
        xs.append(host(x))
        assert info["eta"] <= 1e-10
    K = D.condensed(pat, v, v.sigma_s)
    assert D.backward_errors(K, xs[0], v.b)["eta"] <= 1e-10
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    checks.assert_well_conditioned(xs[0], xo)
    assert np.array_equal(xs[0], xs[1])


def test_hykkt_larger_system(kkt):
    """HyKKT on a 200-stage NMPC system (n=7200, m=6400), gamma = 1e7: eta on
    the 2x2 system <= 1e-10, forward error <= 1e-8 against the saddle-point
    LDL^T, CG iteration count within one of the oracle's."""
    pat = kktgen.nmpc_pattern(200, 32, 4)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(96, 0, 0), 1e-2, 1e2)
    print(f"hykkt n={pat.n} m={pat.m}", flush=True)
    dx0, dy0, inn, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
    assert ok and inn == (pat.n, 0, pat.m)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=200)
    assert info["status"] == 0
    dxh, dyh = host(dx), host(dy)
    check_device_eta(info, D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g))
    assert D.forward_error(dxh, dx0) <= 1e-8 and D.forward_error(dyh, dy0) <= 1e-8
    _, _, oinfo = S.hykkt_cg_solve(pat, v, v.f, v.g, 1e7, tol=1e-10)
    assert abs(info["iters"] - oinfo["iters"]) <= 1


@pytest.mark.parametrize("inst", [0, 1, 2])
def test_hykkt_wide_sigma(kkt, inst):
    """HyKKT on the small NMPC pattern with the late-iteration range
    Sigma_x ~ logU[1e-8, 1e8], gamma = 1e7 (section "Solution 2: HyKKT"):
    the saddle system's condition number is ~1e15, yet CG converges (the
    Schur spectrum 1/(gamma + 1/lambda(S_0)) stays clustered) and (dx, dy)
    match Bunch-Kaufman on the saddle system to 1e-7, eta <= 1e-10 on it, CG
    count within two of the oracle's."""
    pat, _ = kktgen.small_config()
    v = kktgen.nmpc_values(pat, kktgen.rng_for(2, inst, 9), 1e-8, 1e8)
    print(f"hykkt wide sigma inst={inst}", flush=True)
    dxb, dyb, inn = D.hykkt_solution(pat, v, v.f, v.g, 0.0)
    assert inn == (pat.n, 0, pat.m)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=1000)
    assert info["status"] == 0, info
    dxh, dyh = host(dx), host(dy)
    be = D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g)
    assert be["eta"] <= 1e-10
    check_device_eta(info, be)
    assert D.forward_error(dxh, dxb) <= 1e-7 and D.forward_error(dyh, dyb) <= 1e-7
    _, _, oinfo = S.hykkt_cg_solve(pat, v, v.f, v.g, 1e7, tol=1e-10, maxit=1000)
    assert oinfo["status"] == "ok" and abs(info["iters"] - oinfo["iters"]) <= 2, (info, oinfo)


def test_hykkt_paper_scale_cg_count(kkt):
    """HyKKT on the distillation-shaped system at paper scale (n=142,000,
    Sigma_x ~ logU[1e-2, 1e2], gamma = 1e7, tol 1e-10) with the benchmark's
    symbolic options: for three value sets the CG iteration count is within
    one of the oracle's (Cholesky of K_gamma in stage order + the same CG),
    eta on the 2x2 system <= 1e-10, and dx, dy within 1e-6 of the saddle-point
    LDL^T (the two oracle routes differ by 8e-8 there)."""
    pat, _ = kktgen.paper_config()
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=417, max_super=96))
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    for vs in range(3):
        v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, vs), 1e-2, 1e2)
        print(f"paper-scale hykkt value set {vs}", flush=True)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
        info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=200)
        assert info["status"] == 0, info
        dxh, dyh = host(dx), host(dy)
        _, _, oinfo = S.hykkt_cg_solve(pat, v, v.f, v.g, 1e7, tol=1e-10, maxit=200)
        print(vs, info, oinfo, flush=True)
        assert oinfo["status"] == "ok" and abs(info["iters"] - oinfo["iters"]) <= 1
        check_device_eta(info, D.hykkt_backward_errors(pat, v, dxh, dyh, v.f, v.g))
        dx0, dy0, _, ok = S.hykkt_saddle_solve(pat, v, v.f, v.g)
        assert ok and D.forward_error(dxh, dx0) <= 1e-6 and D.forward_error(dyh, dy0) <= 1e-6


def test_hykkt_paper_scale_wide_sigma_eta_stop(kkt):
    """HyKKT at paper scale (n=142,000) in the late-iteration range
    Sigma_x ~ logU[1e-8, 1e8], gamma = 1e7 (section "Solution 2: HyKKT").
    There lambda_min(J K0^{-1} J^T) is ~1e-11, so kappa(S_gamma) is in the
    thousands and CG cannot bring ||r|| below 1e-10 ||c|| (the oracle's CG
    stalls too); the saddle system's normwise backward error, the gate, falls
    below 1e-10 within tens of iterations. With eta_tol = 1e-10 the CG stops
    on its bound: the library's eta and the oracle's evaluation of the same
    (dx, dy) are both <= 1e-10 for two value sets."""
    pat, _ = kktgen.paper_config()
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=417, max_super=96))
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    dy = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    for vs in range(2):
        v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, vs), 1e-8, 1e8)
        print(f"paper-scale hykkt wide sigma value set {vs}", flush=True)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
        assert f.status()[0] == 0
        info = f.cg_schur(dev(v.f), dev(v.g), dx, dy, tol=1e-10, maxit=300, eta_tol=1e-10)
        print(vs, info, flush=True)
        assert info["status"] == 0 and info["eta_stop"] == 1, info
        be = D.hykkt_backward_errors(pat, v, host(dx), host(dy), v.f, v.g)
        check_device_eta(info, be)


@pytest.mark.parametrize("h2", [40, 100], ids=["fused-update", "tile-update"])
def test_front_with_many_children(kkt, h2):
    """Five branches coupled to a hub coupled to a root block, natural order,
    supernodes of at most 24 columns and no amalgamation: the hub's front
    has five children and an update part of h2 rows, so the children's
    pass-through entries take the path for more than two children, in the
    front kernel's epilogue (40 rows) and in the tile update kernel (100
    rows, a level of one front). eta <= 1e-10 and forward error <= 1e-8
    against the oracle (Sigma in [1e-2, 1e2]); the queue schedule bitwise
    equal to the level schedule."""
    pat = kktgen.hub_pattern(5, 20, 24, h2)
    v = kktgen.hub_values(pat, kktgen.rng_for(96, 0, 0), 1e-2, 1e2)
    sym = kkt.Symbolic.from_pattern(pat, ordering=kkt.ORDER_NATURAL, max_super=24, relax_small=-1, relax_frac=0.0)
    cp, par, nr = sym.supernodes()
    nch = np.bincount(par[par >= 0], minlength=len(par))
    hub = int(nch.argmax())
    print(f"hub front: {nch[hub]} children, {nr[hub]} rows, {cp[hub + 1] - cp[hub]} columns", flush=True)
    assert nch[hub] == 5 and nr[hub] - (cp[hub + 1] - cp[hub]) == h2
    xs = []
    for sched in (kkt.SCHEDULE_LEVELS, kkt.SCHEDULE_QUEUE):
        f = kkt.Factor(sym)
        f.set_schedule(sched)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        assert f.status()[0] == 0
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info = f.solve(dev(v.b), x)
        assert info["eta"] <= 1e-10
        xs.append(host(x))
    K = D.condensed(pat, v, v.sigma_s)
    assert D.backward_errors(K, xs[0], v.b)["eta"] <= 1e-10
    xo, oinfo = S.lifted_solve(pat, v, v.b)
    assert oinfo["spd"]
    checks.assert_well_conditioned(xs[0], xo)
    assert np.array_equal(xs[0], xs[1])


@pytest.mark.parametrize("nd", [True, False], ids=["nd", "natural"])
def test_update_split_bitwise(kkt, nd):
    """The launch shape of the update matrices (every level in the front's
    workgroup, the default split, every level by tiles) changes no bit of
    the solution, for a plain factor and for a batch; eta <= 1e-10."""
    pat = kktgen.distillation_pattern(40)
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 40, 0), 1e-8, 1e8)
    opts = dict(ordering=2, nd_leaf=200) if nd else dict(ordering=1)
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    xs = []
    for split in ((0, 0), (48, 96), (1 << 30, 0)):
        f = kkt.Factor(sym)
        f.set_update_split(*split)
        f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
        x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info = f.solve(dev(v.b), x)
        assert info["eta"] <= 1e-10, (split, info)
        xs.append(host(x))
        B = kkt.Batch([sym, sym])
        B.set_update_split(*split)
        cat = lambda a: dev(np.concatenate([a, a]))
        B.refactor(cat(v.w_vals), cat(v.j_vals), cat(v.sigma_x), cat(v.sigma_s))
        xb = torch.zeros(2 * pat.n, dtype=torch.float64, device="cuda")
        B.solve(cat(v.b), xb)
        xbh = host(xb)
        assert np.array_equal(xbh[:pat.n], xs[-1]) and np.array_equal(xbh[pat.n:], xs[-1])
    print("update split variants: max |dx|", max(np.abs(a - xs[0]).max() for a in xs), flush=True)
    assert np.array_equal(xs[0], xs[1]) and np.array_equal(xs[0], xs[2])
    with pytest.raises(kkt.KKTError):
        kkt.Factor(sym).set_update_split(-1, 0)


@pytest.mark.parametrize("case", ["distillation-nd", "distillation-natural", "nmpc-batch"])
def test_small_fronts_bitwise(kkt, case):
    """The four-wave front factorization (levels of narrow fronts; fronts of
    at most 208 rows take the fused panel path, taller ones the pivot chain
    plus row-by-row TRSM) changes no bit of the solution against the
    eight-wave one, for a plain factor and for a batch; every level by four
    waves, none, and a threshold in between; eta <= 1e-10."""
    if case == "nmpc-batch":
        shapes = kktgen.batch_shapes(6)
        pats = [kktgen.nmpc_pattern(*sh) for sh in shapes]
        vals = [kktgen.nmpc_values(p, kktgen.rng_for(3, q, 1), 1e-6, 1e6) for q, p in enumerate(pats)]
        syms = [kkt.Symbolic.from_pattern(p, ordering=2, nd_leaf=64, max_super=48) for p in pats]
    else:
        pat = kktgen.distillation_pattern(40)
        v = kktgen.distillation_values(pat, kktgen.rng_for(1, 40, 0), 1e-8, 1e8)
        opts = dict(ordering=2, nd_leaf=200) if case.endswith("nd") else dict(ordering=1)
        pats, vals, syms = [pat], [v], [kkt.Symbolic.from_pattern(pat, **opts)]
    max_rows = max(s.stats()["max_rows"] for s in syms)
    print(f"{case}: {len(syms)} instance(s), fronts up to {max_rows} rows", flush=True)
    xs_plain, xs_batch = [], []
    for small in (0, 48, 1 << 20):
        xp = []
        for pat, v, sym in zip(pats, vals, syms):
            f = kkt.Factor(sym)
            f.set_small_fronts(small)
            f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
            x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
            info = f.solve(dev(v.b), x)
            assert info["eta"] <= 1e-10, (small, info)
            xp.append(host(x))
            f.close()
        xs_plain.append(np.concatenate(xp))
        B = kkt.Batch(syms)
        B.set_small_fronts(small)
        cat = lambda f: dev(np.concatenate([getattr(v, f) for v in vals]))
        B.refactor(cat("w_vals"), cat("j_vals"), cat("sigma_x"), cat("sigma_s"))
        xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
        B.solve(cat("b"), xb)
        xs_batch.append(host(xb))
        B.close()
    for k in range(3):
        assert np.array_equal(xs_plain[k], xs_plain[0]), k
        assert np.array_equal(xs_batch[k], xs_plain[0]), k
    with pytest.raises(kkt.KKTError):
        kkt.Factor(syms[0]).set_small_fronts(-1)
