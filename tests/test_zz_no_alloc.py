"""kkt_solve_noalloc (the allocation-free refined solve) against kkt_solve.

Both run the same kernels in the same order on the same factor, so x must be
the same bit for bit; each result also passes the oracle's backward-error
gate (eta <= 1e-10). Two calls in a row share the static workspace, the
second on a smaller system; the asynchronous form (no info) matches too; a
system whose workspace exceeds the array is refused with BUDGET.
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


def factor_for(kkt, pat, v, **kw):
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, **kw))
    f.refactor(dev(v.w_vals), dev(v.j_vals), dev(v.sigma_x), dev(v.sigma_s))
    assert f.status()[0] == 0
    return f


def test_noalloc_matches_solve(kkt):
    big_pat, _ = kktgen.paper_config(200)
    big_v = kktgen.distillation_values(big_pat, kktgen.rng_for(1, 0, 4), 1e-8, 1e8)
    small_pat = kktgen.nmpc_pattern(30, 8, 1)
    small_v = kktgen.nmpc_values(small_pat, kktgen.rng_for(0, 9, 1), 1e-6, 1e6)
    cases = [("distillation N=200", big_pat, big_v, dict(ordering=2, nd_leaf=128)),
             ("nmpc N=30", small_pat, small_v, dict(ordering=1))]
    for name, pat, v, kw in cases:
        print(f"noalloc vs solve: {name} n={pat.n}", flush=True)
        f = factor_for(kkt, pat, v, **kw)
        b = dev(v.b)
        x_ref = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
        info_ref = f.solve(b, x_ref)
        x_na = torch.full((pat.n,), float("nan"), dtype=torch.float64, device="cuda")
        info_na = f.solve_noalloc(b, x_na)
        xr, xn = host(x_ref), host(x_na)
        assert np.array_equal(xr, xn), name
        assert info_na == info_ref, (info_na, info_ref)
        be = D.backward_errors(D.condensed(pat, v, v.sigma_s), xn, v.b)
        assert info_na["eta"] <= 1e-10 and be["eta"] <= 1e-10, (info_na, be)
        # the asynchronous form
        x_as = torch.full((pat.n,), float("nan"), dtype=torch.float64, device="cuda")
        assert f.solve_noalloc(b, x_as, info=False) is None
        assert f.status()[0] == 0
        assert np.array_equal(host(x_as), xr), name


def test_noalloc_refuses_oversized_workspace(kkt):
    """A diagonal system of 1.5M variables: its three n-vectors alone need
    36 MB, more than the 32 MiB array, so the call is refused before any
    launch."""
    n = 1_500_000
    pat = kktgen.Pattern(n, 0, np.zeros(n + 1, np.int32), np.zeros(0, np.int32),
                         np.zeros(1, np.int32), np.zeros(0, np.int32))
    print(f"noalloc budget refusal n={n}", flush=True)
    f = kkt.Factor(kkt.Symbolic.from_pattern(pat, ordering=1))
    empty = torch.zeros(0, dtype=torch.float64, device="cuda")
    f.refactor(empty, empty, torch.ones(n, dtype=torch.float64, device="cuda"), empty)
    assert f.status()[0] == 0
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(kkt.KKTError) as e:
        f.solve_noalloc(torch.ones(n, dtype=torch.float64, device="cuda"), x)
    assert e.value.status == 9 and "scratch" in str(e.value)
