"""Inertia correction, slack / multiplier recovery and refinement on the full
(augmented) system, through the C ABI, against the FP64 oracle.

Tolerances:
  * augmented solve, Sigma in [1e-2, 1e2]: (dx, ds, dz) each within a
    relative forward error of 1e-8 of Bunch-Kaufman on the explicit augmented
    system of eq. (kkt:augmented), entry by entry as in tests/checks.py; the
    normwise backward error eta <= 1e-10 by the oracle's evaluator, and the
    library's own eta within a factor of 2 (or 1e-15) of it;
  * Sigma ~ logU[1e-8, 1e8]: eta <= 1e-10 (the forward error is bounded by
    the conditioning only);
  * inertia correction: the accepted delta and the number of trials equal the
    oracle's (whose decisions come from the inertia of the regularised
    augmented system, Bunch-Kaufman), and K + delta I x = b is solved to a
    forward error of 1e-8 against numpy.
"""
import numpy as np
import pytest

import checks
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


def augmented_run(kkt, pat, v, r1, r2, r4, **kw):
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, **kw))
    f.keep_augmented(True)
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    assert f.status()[0] == 0
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    ds = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    dz = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    info = f.solve_augmented(dev(r1), dev(r2), dev(r4), dx, ds, dz)
    return info, host(dx), host(ds), host(dz), f


def rhs(pat, seed):
    rng = kktgen.rng_for(96, seed, 0)
    return rng.standard_normal(pat.n), rng.standard_normal(pat.m), rng.standard_normal(pat.m)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_augmented_matches_oracle(kkt, seed):
    pat, v = kktgen.workload("small", instance=seed)
    r1, r2, r4 = rhs(pat, seed)
    print(f"augmented small seed={seed}", flush=True)
    info, dx, ds, dz, _ = augmented_run(kkt, pat, v, r1, r2, r4, ordering=2, nd_leaf=64)
    assert info["status"] == 0, info
    A = D.lifted_augmented(pat, v)
    p = -np.concatenate([r1, r2, r4])
    zs = D.bunch_kaufman(A).solve(p)
    n, m = pat.n, pat.m
    checks.assert_well_conditioned(dx, zs[:n], "dx")
    checks.assert_well_conditioned(ds, zs[n:n + m], "ds")
    checks.assert_well_conditioned(dz, zs[n + m:], "dz")
    be = D.backward_errors(A, np.concatenate([dx, ds, dz]), p)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15), (info, be)
    # the condensation and recovery identities (stated after eq. (kkt:condensed))
    K = D.condensed(pat, v, v.sigma_s).toarray()
    dxc = np.linalg.solve(K, D.condensed_rhs(pat, v, r1, r2, r4))
    dsc, dzc = D.recover_slack_steps(pat, v, dxc, r2, r4)
    checks.assert_well_conditioned(dx, dxc, "dx condensed")
    checks.assert_well_conditioned(ds, dsc, "ds recovered")
    checks.assert_well_conditioned(dz, dzc, "dz recovered")


def test_augmented_wide_sigma(kkt):
    """Sigma ~ logU[1e-8, 1e8] (late interior-point iterations): the
    augmented system is badly scaled, the refinement on it keeps its
    backward error at the FP64 level."""
    pat, _ = kktgen.workload("small", instance=4)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 4, 5), 1e-8, 1e8)
    r1, r2, r4 = rhs(pat, 7)
    print("augmented wide sigma", flush=True)
    info, dx, ds, dz, _ = augmented_run(kkt, pat, v, r1, r2, r4, ordering=1)
    A = D.lifted_augmented(pat, v)
    p = -np.concatenate([r1, r2, r4])
    be = D.backward_errors(A, np.concatenate([dx, ds, dz]), p)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10, (info, be)
    assert abs(info["eta"] - be["eta"]) <= max(0.5 * be["eta"], 1e-15), (info, be)


def indefinite_case():
    pat = kktgen.nmpc_pattern(10, 4, 1)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(95, 0, 0), 1e-2, 1e2)
    K = D.condensed(pat, v, v.sigma_s).toarray()
    s = pat.meta["stage"]
    v.sigma_x[3 * s:4 * s] -= 30.0 + np.linalg.eigvalsh(K).max()
    return pat, v


def test_inertia_correction_matches_oracle(kkt):
    pat, v = indefinite_case()
    print("inertia correction", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=1))
    dv = [dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s)]
    f.refactor(*dv)
    assert f.status()[0] == 4  # NOT_SPD without correction
    info = f.refactor_inertia(*dv)
    delta, trials, last = D.inertia_correction(pat, v)
    assert info["status"] == 0 and info["delta"] == delta and info["trials"] == len(trials), (info, trials)
    K = D.condensed(pat, v, v.sigma_s).toarray() + delta * np.eye(pat.n)
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    si = f.solve(dev(v.b), x)
    assert si["eta"] <= 1e-10
    assert D.forward_error(host(x), np.linalg.solve(K, v.b)) <= 1e-8
    # the factor remembers delta: the next correction starts from delta / 3
    info2 = f.refactor_inertia(*dv)
    delta2, trials2, _ = D.inertia_correction(pat, v, delta_last=last)
    assert info2["status"] == 0 and info2["delta"] == pytest.approx(delta2, rel=1e-15)
    assert info2["trials"] == len(trials2), (info2, trials2)
    # a definite matrix needs no delta
    pat0, v0 = kktgen.workload("small", instance=1)
    f0 = kkt.Factor(kkt.Symbolic.from_pattern(pat0))
    i0 = f0.refactor_inertia(dev(v0.w_vals), dev(v0.j_vals), dev(v0.sigma_x), dev(v0.sigma_s))
    assert i0 == dict(status=0, trials=1, delta=0.0)
    # an upper bound below the needed delta: NOT_SPD
    fb = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=1))
    o = kkt.kkt_inertia_opts_default()
    o.delta_max = 1.0
    ib = fb.refactor_inertia(*dv, opts=o)
    assert ib["status"] == 4 and fb.status()[0] == 4


def test_inertia_correction_then_augmented(kkt):
    """The corrected factor solves the regularised augmented system (delta on
    the Hessian block), checked against Bunch-Kaufman on it."""
    pat, v = indefinite_case()
    print("inertia correction + augmented", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=16))
    f.keep_augmented(True)
    info = f.refactor_inertia(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    assert info["status"] == 0 and info["delta"] > 0
    r1, r2, r4 = rhs(pat, 3)
    dx = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    ds = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    dz = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    ai = f.solve_augmented(dev(r1), dev(r2), dev(r4), dx, ds, dz)
    A = D.lifted_augmented_regularized(pat, v, info["delta"])
    p = -np.concatenate([r1, r2, r4])
    z = np.concatenate([host(dx), host(ds), host(dz)])
    be = D.backward_errors(A, z, p)
    assert be["eta"] <= 1e-10 and ai["eta"] <= 1e-10, (ai, be)
    assert D.forward_error(z, D.bunch_kaufman(A).solve(p)) <= 1e-8


def general_case(n=300):
    pat = kktgen.general_pattern(kktgen.rng_for(97, n, 0), n, (2 * n) // 3, 0.02, hub_cols=2)
    return pat, kktgen.general_values(pat, kktgen.rng_for(97, n, 1), 1e-2, 1e2)


def test_general_pattern_augmented_and_inertia(kkt):
    """Unstructured pattern: the augmented solve against Bunch-Kaufman on the
    3x3 system; then Sigma_x made strongly negative on a random tenth of the
    variables (K indefinite), the inertia correction's delta and trial count
    equal the oracle's and the corrected factor solves K + delta I."""
    pat, v = general_case()
    r1, r2, r4 = rhs(pat, 11)
    print(f"general augmented n={pat.n} m={pat.m}", flush=True)
    info, dx, ds, dz, _ = augmented_run(kkt, pat, v, r1, r2, r4, ordering=2, nd_leaf=64)
    assert info["status"] == 0, info
    A = D.lifted_augmented(pat, v)
    p = -np.concatenate([r1, r2, r4])
    zs = D.bunch_kaufman(A).solve(p)
    n, m = pat.n, pat.m
    checks.assert_well_conditioned(dx, zs[:n], "dx")
    checks.assert_well_conditioned(ds, zs[n:n + m], "ds")
    checks.assert_well_conditioned(dz, zs[n + m:], "dz")
    be = D.backward_errors(A, np.concatenate([dx, ds, dz]), p)
    assert be["eta"] <= 1e-10 and info["eta"] <= 1e-10
    # indefinite K
    K = D.condensed(pat, v, v.sigma_s).toarray()
    neg = kktgen.rng_for(97, n, 2).choice(n, n // 10, replace=False)
    v.sigma_x[neg] -= 30.0 + np.linalg.eigvalsh(K).max()
    print("general inertia correction", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    dv = [dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s)]
    f.refactor(*dv)
    assert f.status()[0] == 4  # NOT_SPD without correction
    ic = f.refactor_inertia(*dv)
    delta, trials, _ = D.inertia_correction(pat, v)
    assert ic["status"] == 0 and ic["delta"] == delta and ic["trials"] == len(trials), (ic, trials)
    Kd = D.condensed(pat, v, v.sigma_s).toarray() + delta * np.eye(n)
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    si = f.solve(dev(v.b), x)
    assert si["eta"] <= 1e-10
    assert D.forward_error(host(x), np.linalg.solve(Kd, v.b)) <= 1e-8


def test_augmented_refused_on_hykkt_factor(kkt):
    pat, v = kktgen.workload("hykkt")
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), None, 1e7)
    z = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    zm = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError) as e:
        f.solve_augmented(z, zm, zm, z.clone(), zm.clone(), zm.clone())
    assert e.value.status == 3


def test_augmented_needs_kept_values(kkt):
    """Without kkt_factor_keep_augmented the Lifted-KKT refactor keeps no
    copies, and the augmented solve is refused (STATE)."""
    pat, v = kktgen.workload("small", instance=2)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    z = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    zm = torch.zeros(pat.m, dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError) as e:
        f.solve_augmented(z, zm, zm, z.clone(), zm.clone(), zm.clone())
    assert e.value.status == 3
