"""Host-side checks of libkkt through its C ABI (no GPU calls).

  * the shared library loads and exports every function include/*.h declares;
  * the symbolic analysis matches brute-force boolean elimination (column
    structure of L under the library's own ordering), on the pinned small
    pattern and on random patterns;
  * the ordering is a permutation and the supernode tree is postordered;
  * malformed input returns the documented status codes.
"""
import glob
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import kktgen
from oracle import symbolic as Y

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def kkt():
    from paper_2403_15913_amd import kkt as K
    if not os.path.exists(K.LIB_PATH):
        from paper_2403_15913_amd import build
        build.build()
    K.lib()
    return K


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(kkt_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_exports_every_declared_symbol(kkt):
    names = declared_functions()
    assert len(names) >= 15
    lib = kkt.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every exported entry point under its C name
    assert set(names) <= set(kkt.SIGNATURES), set(names) - set(kkt.SIGNATURES)


def test_status_strings(kkt):
    for code, name in kkt.STATUS_NAMES.items():
        assert kkt.lib().kkt_status_string(code).decode() == name


def brute_force_nnz(pat, perm):
    L = Y.cholesky_structure(Y.k_pattern(pat), perm)
    return Y.stats(L)


def test_pinned_small_pattern(kkt):
    pat, _ = kktgen.small_config()
    s = kkt.Symbolic.from_pattern(pat, ordering=kkt.ORDER_NATURAL, max_super=1, relax_small=-1, relax_frac=0.0)
    st_ = s.stats()
    assert (st_["nnz_k"], st_["nnz_l_exact"], st_["flops_exact"]) == (3720, 4749, 50657)
    assert st_["nnz_l"] == 4749 and st_["nsuper"] == pat.n
    # natural stage order is already an elimination-tree postorder for this chain
    assert np.array_equal(s.perm(), np.arange(pat.n))


@pytest.mark.parametrize("kw", [dict(ordering=1), dict(ordering=2, nd_leaf=64), dict(ordering=2, nd_leaf=16),
                                dict(ordering=0)])
def test_structure_matches_brute_force(kkt, kw):
    pat, _ = kktgen.small_config()
    s = kkt.Symbolic.from_pattern(pat, **kw)
    st_ = s.stats()
    perm = s.perm()
    assert np.array_equal(np.sort(perm), np.arange(pat.n))
    bf = brute_force_nnz(pat, perm)
    assert st_["nnz_l_exact"] == bf["nnz_l"] and st_["flops_exact"] == bf["sum_c2"]
    check_supernodes(s, bf, pat.n)


def check_supernodes(s, bf, n):
    st_ = s.stats()
    cp, par, nr = s.supernodes()
    ns = st_["nsuper"]
    assert cp[0] == 0 and cp[-1] == n and (np.diff(cp) > 0).all()
    ncol = np.diff(cp)
    assert ncol.max() == st_["max_cols"] and nr.max() == st_["max_rows"]
    for q in range(ns):
        assert par[q] == -1 or par[q] > q
        # a front holds at least the exact structure of its first column
        assert nr[q] >= bf["counts"][cp[q]]
        assert nr[q] >= ncol[q]
        if par[q] == -1:
            assert nr[q] == ncol[q]
    stored = int((nr.astype(np.int64) * ncol - ncol * (ncol - 1) // 2).sum())
    assert stored == st_["nnz_l"] >= st_["nnz_l_exact"]


def test_nested_dissection_reduces_depth(kkt):
    pat = kktgen.distillation_pattern(64)
    nat = kkt.Symbolic.from_pattern(pat, ordering=kkt.ORDER_NATURAL).stats()
    nd = kkt.Symbolic.from_pattern(pat, ordering=kkt.ORDER_ND, nd_leaf=300).stats()
    assert nd["levels"] * 3 < nat["levels"]
    assert nd["nnz_l_exact"] <= 3 * nat["nnz_l_exact"]


@st.composite
def random_pattern(draw):
    n = draw(st.integers(1, 40))
    m = draw(st.integers(0, 30))
    rng = np.random.default_rng(draw(st.integers(0, 2**31 - 1)))
    dens = draw(st.floats(0.02, 0.3))
    w_rows = [np.sort(np.unique(np.append(rng.choice(i + 1, size=rng.binomial(i + 1, dens), replace=False), i)))
              for i in range(n)]
    j_rows = [np.sort(rng.choice(n, size=min(n, rng.integers(0, 5)), replace=False)) for _ in range(m)]
    wr = np.concatenate([[0], np.cumsum([len(r) for r in w_rows])]).astype(np.int32)
    jr = np.concatenate([[0], np.cumsum([len(r) for r in j_rows])]).astype(np.int32)
    wc = np.concatenate(w_rows).astype(np.int32) if n else np.zeros(0, np.int32)
    jc = np.concatenate(j_rows).astype(np.int32) if m and jr[-1] else np.zeros(0, np.int32)
    return kktgen.Pattern(n, m, wr, wc, jr, jc, {})


@settings(max_examples=60, deadline=None)
@given(pat=random_pattern(), ordering=st.sampled_from([1, 2]), leaf=st.sampled_from([1, 3, 8]),
       max_super=st.sampled_from([1, 4, 96]))
def test_random_patterns(kkt, pat, ordering, leaf, max_super):
    s = kkt.Symbolic.from_pattern(pat, ordering=ordering, nd_leaf=leaf, max_super=max_super)
    perm = s.perm()
    assert np.array_equal(np.sort(perm), np.arange(pat.n))
    bf = brute_force_nnz(pat, perm)
    st_ = s.stats()
    assert st_["nnz_l_exact"] == bf["nnz_l"]
    check_supernodes(s, bf, pat.n)
    assert st_["max_cols"] <= max_super


def status_of(kkt, *args, opt=None):
    try:
        kkt.kkt_symbolic_analyze(*args, opt=opt)
        return 0
    except kkt.KKTError as e:
        return e.status


def test_error_codes(kkt):
    n, m = 3, 1
    wr, wc = np.array([0, 1, 2, 3]), np.array([0, 1, 2])
    jr, jc = np.array([0, 2]), np.array([0, 2])
    assert status_of(kkt, n, m, wr, wc, jr, jc) == 0
    assert status_of(kkt, n, m, wr, np.array([0, 2, 2]), jr, jc) == 2           # W entry above the diagonal
    assert status_of(kkt, n, m, np.array([0, 1, 3, 3]), np.array([0, 1, 0]), jr, jc) == 2  # unsorted W row
    assert status_of(kkt, n, m, wr, wc, jr, np.array([2, 0])) == 2              # unsorted J row
    assert status_of(kkt, n, m, wr, wc, jr, np.array([0, 3])) == 2              # J column out of range
    assert status_of(kkt, n, m, np.array([1, 1, 2, 3]), wc, jr, jc) == 2        # row pointer not at 0
    assert status_of(kkt, -1, m, wr, wc, jr, jc) == 1                           # negative size
    bad = kkt.Options(7, 0, 0, 0, -1.0)
    assert status_of(kkt, n, m, wr, wc, jr, jc, opt=bad) == 1                   # unknown ordering
    wide = kkt.Options(0, 0, 200, 0, -1.0)
    assert status_of(kkt, n, m, wr, wc, jr, jc, opt=wide) == 1                  # max_super > 128
    neg = kkt.Options(0, 0, 0, 0, -1.0, -1)
    assert status_of(kkt, n, m, wr, wc, jr, jc, opt=neg) == 1                   # negative front_lds_max
    tiny = kkt.Options(0, 0, 0, 0, -1.0, 1)
    assert status_of(kkt, n, m, wr, wc, jr, jc, opt=tiny) == 0                  # raised to 4 KiB
    import ctypes as C
    assert kkt.lib().kkt_symbolic_analyze(n, m, None, None, None, None, None, None) == 1  # NULL out
    assert kkt.lib().kkt_symbolic_get_stats(None, None) == 1


def test_empty_and_tiny(kkt):
    s = kkt.Symbolic(1, 0, np.array([0, 1]), np.array([0]), np.array([0]), np.zeros(0))
    st_ = s.stats()
    assert st_["nsuper"] == 1 and st_["nnz_l"] == 1
    s = kkt.Symbolic(0, 0, np.array([0]), np.zeros(0), np.array([0]), np.zeros(0))
    assert s.stats()["nsuper"] == 0


def test_stagewise_rejects_bad_stages(kkt):
    """The stage-structured solver checks its stage ranges and the block
    tridiagonal structure on the host, before any device call: INVALID_ARG
    (1) for ranges that do not cover 0 .. n or hold an empty stage, PATTERN
    (2) for a stage wider than 80 or a K position coupling stages two apart
    (a split of each NMPC stage into states and controls puts the dynamics
    rows x_{k+1} - A x_k - B u_k across three sub-stages)."""
    import kktgen
    pat = kktgen.nmpc_pattern(6, 8, 1)
    s = kkt.Symbolic.from_pattern(pat)
    st = pat.meta["stage"]

    def code(sp):
        try:
            kkt.Stagewise([s], [np.asarray(sp, dtype=np.int32)])
        except kkt.KKTError as e:
            return e.status
        return 0

    assert code([0, 18, 36]) == 1                                  # does not end at n
    assert code([0, 0, 54]) == 1                                   # empty stage
    assert code([1, 54]) == 1                                      # does not start at 0
    split = [0]
    for k in range(6):
        split += [k * st + 8, (k + 1) * st]
    assert code(split) == 2                                        # states / controls split
    wide = kkt.Symbolic.from_pattern(kktgen.nmpc_pattern(10, 8, 1))
    try:
        kkt.Stagewise([wide], [np.array([0, 90], dtype=np.int32)])  # one stage of 90
        raise AssertionError("accepted a stage of 90")
    except kkt.KKTError as e:
        assert e.status == 2


def test_stagewise_banded_pattern_stage_width(kkt):
    """A band-limited unstructured pattern (entries within 40 of the
    diagonal) is block tridiagonal over stages at least 40 wide; stages of
    30 put entries two stages apart: PATTERN (2) on the host."""
    import kktgen
    pat = kktgen.general_pattern(kktgen.rng_for(8, 0, 0), 2000, 1600, 0.3, row_max=6, band=40)
    s = kkt.Symbolic.from_pattern(pat)
    sp = np.append(np.arange(0, pat.n, 30), pat.n).astype(np.int32)
    try:
        kkt.Stagewise([s], [sp])
        raise AssertionError("accepted stages narrower than the band")
    except kkt.KKTError as e:
        assert e.status == 2


def _front_lds(r, c):
    # LDS of a front panel in the factor and sweep kernels (host layout rule)
    fac = (r | 1) * ((c + 15) // 16 * 16) * 8 + r * 4 + 16
    sol = ((((r | 1) * c + 1) // 2 * 2) + r + c) * 8
    return max(fac, sol)


@pytest.mark.parametrize("budget", [8192, 16 * 1024])
def test_large_fronts_structure(kkt, budget):
    """Fronts too tall for the LDS budget at one column become large fronts
    (at most 64 columns, factored in HBM) instead of failing the analysis;
    the structure still matches brute-force elimination."""
    pat = kktgen.distillation_pattern(6)
    s = kkt.Symbolic.from_pattern(pat, ordering=2, nd_leaf=100, front_lds_max=budget)
    st_ = s.stats()
    bf = brute_force_nnz(pat, s.perm())
    assert st_["nnz_l_exact"] == bf["nnz_l"] and st_["flops_exact"] == bf["sum_c2"]
    check_supernodes(s, bf, pat.n)
    cp, par, nr = s.supernodes()
    ncol = np.diff(cp)
    large = np.array([_front_lds(int(r), int(c)) > budget for r, c in zip(nr, ncol)])
    assert 0 < large.sum() == st_["large_fronts"] <= st_["nsuper"]
    assert (ncol[large] <= 64).all()
    # every other front fits its panel in the budget
    assert all(_front_lds(int(r), int(c)) <= budget for r, c, lg in zip(nr, ncol, large) if not lg)
    if budget == 16 * 1024:
        assert large.sum() < st_["nsuper"]


def test_tall_fronts_under_default_budget(kkt):
    """Stages 700 variables wide give fronts too tall for 158 KiB of LDS at any width."""
    pat = kktgen.nmpc_pattern(4, 700, 4)
    st_ = kkt.Symbolic.from_pattern(pat, ordering=2).stats()
    assert st_["large_fronts"] > 0 and st_["max_rows"] > (158 * 1024) // (16 * 8)
