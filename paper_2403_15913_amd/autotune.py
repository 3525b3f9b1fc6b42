"""Autotuner for the symbolic options and launch schedule that shape the GPU work.

For a pattern (or a batch of patterns) it measures refactor+solve on the
device for a set of candidate options -- ordering (natural stage order or
nested dissection), nested-dissection leaf size, widest supernode, the launch
schedule (one launch per tree level, or the persistent work queue), the
launch shape of the update matrices (which tree levels form them in a launch
of their own, one wave per tile) and the workgroup size of the front
factorization per tree level (four waves for levels of narrow fronts, so
two can share a compute unit, else eight) -- and keeps the fastest candidate whose
solves all pass the backward-error gate. These options decide the supernode
tree the kernels run on: the depth of the dependency chain, the front sizes
(rows x columns of every LDS panel and of the matrix-core tiles), the total
flops, and how the work of each level is spread over the compute units.

Results are cached in a JSON table keyed by a pattern signature, so a
pattern is tuned once and later analyses reuse the choice:

    from paper_2403_15913_amd import autotune
    best = autotune.tune_pattern(pat, vals)            # measure (GPU)
    sym = kkt.Symbolic.from_pattern(pat, **{k: best[k] for k in ("ordering", "nd_leaf", "max_super")})
    f = kkt.Factor(sym); f.set_schedule(best["schedule"]); f.set_update_split(*best["split"])
    f.set_small_fronts(best["small"])

Timing uses the library's own calls; nothing here computes any part of the
solve.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import kkt

DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_table.json")
ETA_GATE = 1e-10


def signature(pat) -> str:
    """Stable key of a sparsity pattern (sizes + a hash of the index arrays)."""
    h = hashlib.sha1()
    for a in (pat.w_rowptr, pat.w_colind, pat.j_rowptr, pat.j_colind):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    return f"n{pat.n}-m{pat.m}-w{pat.nnz_w}-j{pat.nnz_j}-{h.hexdigest()[:16]}"


def candidates(n: int):
    """Option sets to try for a pattern of n variables: natural order, and
    nested dissection with leaf parts from n/1024 to n/128 vertices (the
    leaf size trades the depth of the chains inside the leaves against the
    number of separator levels)."""
    out = [dict(ordering=kkt.ORDER_NATURAL, nd_leaf=0, max_super=96)]
    for leaf in sorted({max(64, n // k) for k in (1024, 512, 340, 256, 128)}):
        if leaf < n:
            out.append(dict(ordering=kkt.ORDER_ND, nd_leaf=int(leaf), max_super=96))
    # narrower supernodes at the middle leaf size: smaller fronts and panels
    leaf = max(64, n // 340)
    if leaf < n:
        out += [dict(ordering=kkt.ORDER_ND, nd_leaf=int(leaf), max_super=ms) for ms in (64, 48)]
    return out


def load_table(path: str = DEFAULT_TABLE) -> dict:
    if os.path.exists(path):
        with open(path) as fh:
            return json.load(fh)
    return {}


def save_table(table: dict, path: str = DEFAULT_TABLE):
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _dev(a):
    import torch
    return torch.tensor(np.asarray(a), dtype=torch.float64, device="cuda")


# launch shapes of the update matrices (kkt_factor_set_update_split): the
# default, none split, fewer levels split, every level split
SPLITS = ((140, 64), (0, 0), (48, 96), (1 << 30, 0))
# column thresholds of the four-wave front factorization
# (kkt_factor_set_small_fronts): none, then levels whose widest front has at
# most 32, 48 or 64 columns
SMALLS = (0, 32, 48, 64)


def _time_plain(pat, vals, opts, reps: int, schedule: int = kkt.SCHEDULE_LEVELS, split=SPLITS[0],
                small: int = SMALLS[0]):
    import torch
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    f = kkt.Factor(sym)
    f.set_schedule(schedule)
    f.set_update_split(*split)
    f.set_small_fronts(small)
    d = [_dev(vals.w_vals), _dev(vals.j_vals), _dev(vals.sigma_x), _dev(vals.sigma_s)]
    b = _dev(vals.b)
    x = torch.zeros(pat.n, dtype=torch.float64, device="cuda")
    f.refactor(*d)
    f.solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for _ in range(reps):
        f.refactor(*d)
        worst = max(worst, f.solve(b, x)["eta"])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, worst, sym.stats()


def analyze_many(pats, threads: int = 16, **opts):
    """Symbolic analyses of many patterns on host threads (the C call drops the GIL)."""
    with ThreadPoolExecutor(max_workers=max(1, min(threads, len(pats)))) as ex:
        return list(ex.map(lambda p: kkt.Symbolic.from_pattern(p, **opts), pats))


def _time_batch(B, cat, b, x, reps: int):
    import torch
    B.refactor(*cat)
    B.solve(b, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    worst = 0.0
    for _ in range(reps):
        B.refactor(*cat)
        worst = max(worst, max(i["eta"] for i in B.solve(b, x)))
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, worst


def tune_pattern(pat, vals, reps: int = 3, table_path: str | None = DEFAULT_TABLE, force: bool = False,
                 log=None, schedules=(kkt.SCHEDULE_LEVELS,)) -> dict:
    """Best options for one pattern (measured on the GPU, cached by signature).

    The symbolic candidates are timed under the level schedule; then the best
    few are timed again under every schedule in `schedules`, and the fastest
    option set under the level schedule with every launch shape in SPLITS and
    then every threshold in SMALLS. The result holds the symbolic options and
    the "schedule", "split" and "small" entries."""
    key = signature(pat)
    table = load_table(table_path) if table_path else {}
    if not force and key in table:
        return dict(table[key]["options"])
    results = []
    for opts in candidates(pat.n):
        try:
            t, eta, st = _time_plain(pat, vals, opts, reps)
        except kkt.KKTError as e:
            if log:
                log(f"{opts}: {e}")
            continue
        results.append((t, eta, dict(opts, schedule=kkt.SCHEDULE_LEVELS, split=SPLITS[0], small=SMALLS[0]), st))
        if log:
            log(f"{opts}: {1e3 * t:.3f} ms, eta {eta:.1e}, levels {st['levels']}, flops {st['flops']:.3g}")
    # other schedules for the three fastest option sets
    top = sorted((r for r in results if r[1] <= ETA_GATE), key=lambda r: r[0])[:3]
    for sched in schedules:
        if sched == kkt.SCHEDULE_LEVELS:
            continue
        for _, _, o, _ in top:
            opts = {k: o[k] for k in ("ordering", "nd_leaf", "max_super")}
            t, eta, st = _time_plain(pat, vals, opts, reps, sched)
            results.append((t, eta, dict(opts, schedule=sched, split=SPLITS[0], small=SMALLS[0]), st))
            if log:
                log(f"{opts} schedule {sched}: {1e3 * t:.3f} ms, eta {eta:.1e}")
    # launch shapes of the update matrices for the fastest option set
    if top:
        opts = {k: top[0][2][k] for k in ("ordering", "nd_leaf", "max_super")}
        best_split, t_split = SPLITS[0], top[0][0]
        for split in SPLITS[1:]:
            t, eta, st = _time_plain(pat, vals, opts, reps, kkt.SCHEDULE_LEVELS, split)
            results.append((t, eta, dict(opts, schedule=kkt.SCHEDULE_LEVELS, split=split, small=SMALLS[0]), st))
            if log:
                log(f"{opts} split {split}: {1e3 * t:.3f} ms, eta {eta:.1e}")
            if eta <= ETA_GATE and t < t_split:
                best_split, t_split = split, t
        # workgroup size of the front factorization, at the fastest split
        for small in SMALLS[1:]:
            t, eta, st = _time_plain(pat, vals, opts, reps, kkt.SCHEDULE_LEVELS, best_split, small)
            results.append((t, eta, dict(opts, schedule=kkt.SCHEDULE_LEVELS, split=best_split, small=small), st))
            if log:
                log(f"{opts} split {best_split} small {small}: {1e3 * t:.3f} ms, eta {eta:.1e}")
    ok = [r for r in results if r[1] <= ETA_GATE]
    if not ok:
        raise RuntimeError("no candidate passed the backward-error gate")
    t, eta, best, st = min(ok, key=lambda r: r[0])
    if table_path:
        table[key] = dict(options=best, ms=1e3 * t, eta=eta,
                          tried=[dict(options=o, ms=1e3 * tt) for tt, _, o, _ in results])
        save_table(table, table_path)
    return dict(best)


def batch_candidates(nmax: int):
    out = [dict(ordering=kkt.ORDER_NATURAL, nd_leaf=0, max_super=96),
           dict(ordering=kkt.ORDER_NATURAL, nd_leaf=0, max_super=64)]
    out += [dict(ordering=kkt.ORDER_ND, nd_leaf=leaf, max_super=96) for leaf in (256, 1024) if leaf < nmax]
    # narrower supernodes: smaller fronts, so more of them share a compute unit
    out += [dict(ordering=kkt.ORDER_ND, nd_leaf=256, max_super=ms) for ms in (64, 48) if 256 < nmax]
    out += [dict(ordering=kkt.ORDER_ND, nd_leaf=leaf, max_super=48) for leaf in (512, 1024) if leaf < nmax]
    return out


def tune_batch(pats, vals, reps: int = 2, log=None, threads: int = 16) -> dict:
    """One option set and schedule for a whole batch (measured as batched refactor + solve)."""
    import torch
    nmax = max(p.n for p in pats)
    cat = [_dev(np.concatenate([getattr(v, f) for v in vals])) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s")]
    b = _dev(np.concatenate([v.b for v in vals]))
    x = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device="cuda")
    tried = []
    # every option set under the level schedule with each workgroup-size
    # threshold, and under the queue schedule (eight-wave fronts only)
    for opts in batch_candidates(nmax):
        syms = analyze_many(pats, threads, **opts)
        B = kkt.Batch(syms)
        for sched, small in [(kkt.SCHEDULE_LEVELS, sm) for sm in SMALLS] + [(kkt.SCHEDULE_QUEUE, SMALLS[0])]:
            B.set_schedule(sched)
            B.set_small_fronts(small)
            t, eta = _time_batch(B, cat, b, x, reps)
            tried.append((t, eta, dict(opts, schedule=sched, small=small)))
            if log:
                log(f"{opts} schedule {sched} small {small}: {1e3 * t:.3f} ms, eta {eta:.1e}")
        B.close()
    ok = [r for r in tried if r[1] <= ETA_GATE]
    if not ok:
        raise RuntimeError("no candidate passed the backward-error gate")
    t, eta, best = min(ok, key=lambda r: r[0])
    best = dict(best, split=SPLITS[0])
    # launch shapes of the update matrices for the fastest option set
    if best["schedule"] == kkt.SCHEDULE_LEVELS:
        opts = {k: best[k] for k in ("ordering", "nd_leaf", "max_super")}
        B = kkt.Batch(analyze_many(pats, threads, **opts))
        B.set_small_fronts(best["small"])
        for split in SPLITS[1:]:
            B.set_update_split(*split)
            ts, eta = _time_batch(B, cat, b, x, reps)
            tried.append((ts, eta, dict(opts, schedule=kkt.SCHEDULE_LEVELS, small=best["small"], split=split)))
            if log:
                log(f"{opts} small {best['small']} split {split}: {1e3 * ts:.3f} ms, eta {eta:.1e}")
            if eta <= ETA_GATE and ts < t:
                t, best = ts, dict(opts, schedule=kkt.SCHEDULE_LEVELS, small=best["small"], split=split)
        B.close()
    return dict(best=best, ms=1e3 * t, tried=[dict(options=o, ms=round(1e3 * tt, 3)) for tt, _, o in tried])
