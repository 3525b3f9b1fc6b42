"""The interior-point outer loop (kkt_ipm_qp) on synthetic convex LQ-MPC QPs,
through the C ABI, against the oracle's interior-point method (same
algorithm, CPU, sparse LDL^T for the Newton steps).

Tolerances: the same number of iterations (within one); the solution x, s
and z within 1e-6 (relative, inf-norm) of the oracle's; the QP's KKT
conditions met at the GPU's answer (stationarity and feasibility <= 1e-8
relative, z > 0, s > 0, complementarity gap <= 1e-8).
"""
import numpy as np
import pytest

import kktgen
from oracle import ipm

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


def qp_case(name):
    if name.startswith("general"):
        # unstructured W and J (diagonally dominant W, random J rows with shared columns)
        n, m, dens, hubs = (300, 200, 0.02, 2) if name == "general300" else (1500, 1200, 0.003, 3)
        pat = kktgen.general_pattern(kktgen.rng_for(7, n, 0), n, m, dens, hub_cols=hubs)
        v = kktgen.general_values(pat, kktgen.rng_for(7, n, 1), 1e-2, 1e2)
        rng = kktgen.rng_for(100, n, 0)
        return pat, v, rng.standard_normal(n), 0.1 + rng.random(m)
    if name == "small":
        pat, v = kktgen.workload("small")
    else:
        pat, _ = kktgen.paper_config(200)
        v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, 0), 1e-2, 1e2)
    rng = kktgen.rng_for(100, 0 if name == "small" else 1, 0)
    c = rng.standard_normal(pat.n)
    u = 0.1 + rng.random(pat.m)
    return pat, v, c, u


@pytest.mark.parametrize("name", ["small", "distillation200", "general300", "general1500"])
def test_ipm_matches_oracle(kkt, name):
    pat, v, c, u = qp_case(name)
    print(f"ipm {name} n={pat.n} m={pat.m}", flush=True)
    W, c, J, u = ipm.qp_from_pattern(pat, v, c, u)
    xo, so, zo, oinfo = ipm.qp_ipm(W, c, J, u, np.zeros(pat.n), u.copy(), np.ones(pat.m), tol=1e-8)
    assert oinfo["status"] == "ok"
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=64))
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    s = dev(u)
    z = torch.ones(pat.m, dtype=torch.float64, device="cuda")
    info = f.ipm_qp(dev(v.w_vals), dev(v.j_vals), dev(c), dev(u), x, s, z, tol=1e-8)
    print(info, oinfo, flush=True)
    assert info["status"] == 0 and abs(info["iterations"] - oinfo["iterations"]) <= 1, (info, oinfo)
    xh, sh, zh = host(x), host(s), host(z)
    for a, b in ((xh, xo), (sh, so), (zh, zo)):
        assert np.abs(a - b).max() <= 1e-6 * (1 + np.abs(b).max())
    Wd = W.tocsr()
    assert np.abs(Wd @ xh + c + J.T @ zh).max() <= 1e-8 * (1 + np.abs(c).max())
    assert (J @ xh - u).max() <= 1e-8 * (1 + np.abs(u).max())
    assert zh.min() > 0 and sh.min() > 0 and (sh @ zh) / pat.m <= 1e-8
