#!/usr/bin/env python3
"""Refactor+solve throughput of the Newton-step KKT solve on one MI355X.

Default workload: the distillation-column-shaped Lifted-KKT system at paper
scale (N=2000 stages of 71 variables: n=142,000, m=140,000; Sigma ~
logU[1e-8, 1e8]), one symbolic analysis, then refactor+solve pairs cycling
through 10 resident value sets. A step is one pass of the whole path:
assembly of K, supernodal Cholesky, forward/backward sweeps and Richardson
refinement. A pair counts only if its normwise backward error is <= 1e-10.

Prints one JSON line (see the contract fields) with a live roofline figure
for the dominant kernel (HIP events around every launch of the timed
region) and the FP64 oracle timed on the host cores as ``cpu_baseline``.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6      # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0        # MI355X HBM3E
ETA_GATE = 1e-10


def parse():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="paper", choices=["paper", "small"])
    ap.add_argument("--value-sets", type=int, default=10)
    ap.add_argument("--cpu-sample", type=int, default=32, help="oracle refactor+solve pairs timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ordering", type=int, default=0)
    ap.add_argument("--nd-leaf", type=int, default=0)
    ap.add_argument("--max-super", type=int, default=96, help="widest supernode (columns)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick ordering / leaf size by measurement (ignored when --ordering or --nd-leaf is set)")
    ap.add_argument("--hykkt", type=int, default=1, help="also time HyKKT (refactor + Schur CG) at paper scale")
    ap.add_argument("--ipm", type=int, default=1, help="also time the interior-point loop on a paper-scale QP")
    ap.add_argument("--stagewise", type=int, default=1, help="also time the stage-structured solver (paper + batch)")
    ap.add_argument("--large-fronts", type=int, default=1, help="also time a pattern whose fronts are too tall for "
                                                                    "LDS (large-front path)")
    ap.add_argument("--small", type=int, default=1, help="also time the small NMPC system (n=450): plain, "
                                                          "one-instance graph and batched")
    ap.add_argument("--small-pairs", type=int, default=1000, help="plain pairs per value set of the small system")
    ap.add_argument("--small-batch", type=int, default=256, help="instances of the small system per batch (0: skip)")
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched workload (0: skip)")
    ap.add_argument("--batch-ordering", type=int, default=2, help="batch ordering when not autotuned")
    ap.add_argument("--batch-nd-leaf", type=int, default=256, help="batch nested-dissection leaf when not autotuned")
    ap.add_argument("--batch-max-super", type=int, default=48, help="batch widest supernode when not autotuned")
    ap.add_argument("--batch-small", type=int, default=64,
                    help="batch four-wave front column threshold when not autotuned")
    ap.add_argument("--batch-autotune", type=int, default=1, help="pick batch options and schedule by measurement")
    ap.add_argument("--graph-rounds", type=int, default=1, help="refinement rounds recorded in the batch graph")
    ap.add_argument("--schedule", dest="schedule_given", default=None, choices=["levels", "queue"],
                    help="plain-solver launch schedule (default: the autotuner's pick, else levels)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run one plain device copy of this many MiB (HBM counter calibration) and exit")
    ap.add_argument("--serve-requests", type=int, default=10000, help="requests per arrival rate of the served "
                                                                        "workload (0: skip)")
    ap.add_argument("--serve-workers", type=int, default=2, help="workers (streams) of the continuous-batching "
                                                                  "server")
    ap.add_argument("--serve-rho", default="0.5,0.8,1.2,2.0", help="arrival rates as fractions of the plain solver's "
                                                                 "capacity (comma-separated)")
    args = ap.parse_args()
    args.schedule = args.schedule_given or "levels"
    return args


def bench_batched(args, kkt, kktgen, torch, dev):
    """Batched NMPC instances: graph-replayed and eager batched refactor+solve vs one plain factor per instance."""
    from paper_2403_15913_amd import autotune
    count = args.batch
    shapes = kktgen.batch_shapes(count)
    pats = [kktgen.nmpc_pattern(*sh) for sh in shapes]
    vals = [kktgen.nmpc_values(p, kktgen.rng_for(3, q, 1), 1e-6, 1e6) for q, p in enumerate(pats)]

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    # options and schedule from the autotuner (measured on this batch), or fixed ones
    t0 = time.perf_counter()
    if args.batch_autotune:
        tuned = autotune.tune_batch(pats, vals, reps=2)
        best = tuned["best"]
    else:
        tuned = None
        best = dict(ordering=args.batch_ordering, nd_leaf=args.batch_nd_leaf, max_super=args.batch_max_super,
                    schedule=kkt.SCHEDULE_LEVELS, small=args.batch_small)
    tune_s = time.perf_counter() - t0
    opts = {k: best[k] for k in ("ordering", "nd_leaf", "max_super")}
    t0 = time.perf_counter()
    syms = autotune.analyze_many(pats, **opts)
    analyze_s = time.perf_counter() - t0
    B = kkt.Batch(syms)
    B.set_schedule(best["schedule"])
    B.set_update_split(*best.get("split", (140, 64)))
    B.set_small_fronts(best.get("small", 0))
    cat = {f: T(np.concatenate([getattr(v, f) for v in vals])) for f in ("w_vals", "j_vals", "sigma_x", "sigma_s", "b")}
    x = torch.zeros(int(B.ofs["n"][-1]), dtype=torch.float64, device=dev)
    reps = 5

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / reps, out

    def eager():
        B.refactor(cat["w_vals"], cat["j_vals"], cat["sigma_x"], cat["sigma_s"])
        return B.solve(cat["b"], x)

    eager_s = {}
    for name, sched in (("levels", kkt.SCHEDULE_LEVELS), ("queue", kkt.SCHEDULE_QUEUE)):
        B.set_schedule(sched)
        eager_s[name], _ = timed(eager)
    B.set_schedule(best["schedule"])
    # per-phase kernel time of the eager batched refactor+solve (HIP events around every launch)
    B.set_timing(True)
    B.read_timing()
    for _ in range(reps):
        eager()
    btm = B.read_timing()
    B.set_timing(False)
    xg = torch.zeros_like(x)
    B.capture(cat["w_vals"], cat["j_vals"], cat["sigma_x"], cat["sigma_s"], cat["b"], xg, rounds=args.graph_rounds)
    tg, infos = timed(B.replay)
    etas = np.array([i["eta"] for i in infos])
    ok = int((etas <= ETA_GATE).sum())
    # plain: one factor per instance, one instance per launch sequence (level schedule)
    facs = [kkt.Factor(s) for s in syms]
    dv = [dict(w=T(v.w_vals), j=T(v.j_vals), sx=T(v.sigma_x), ss=T(v.sigma_s), b=T(v.b)) for v in vals]
    xs = [torch.zeros(p.n, dtype=torch.float64, device=dev) for p in pats]

    def pstep():
        res = []
        for f, d, xq in zip(facs, dv, xs):
            f.refactor(d["w"], d["j"], d["sx"], d["ss"])
            res.append(f.solve(d["b"], xq))
        return res

    pstep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinfos = pstep()
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    pok = int(sum(i["eta"] <= ETA_GATE for i in pinfos))
    # the plain solver also on the analyses it would use by itself (the
    # library's default options), which can be faster one instance at a time
    # than the options tuned for the batch
    facs_d = [kkt.Factor(sd) for sd in autotune.analyze_many(pats)]
    xs_d = [torch.zeros(p.n, dtype=torch.float64, device=dev) for p in pats]

    def pstep_d():
        res = []
        for f, d, xq in zip(facs_d, dv, xs_d):
            f.refactor(d["w"], d["j"], d["sx"], d["ss"])
            res.append(f.solve(d["b"], xq))
        return res

    pstep_d()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pinfos_d = pstep_d()
    torch.cuda.synchronize()
    tp_d = time.perf_counter() - t0
    pok_d = int(sum(i["eta"] <= ETA_GATE for i in pinfos_d))
    for f in facs_d:
        f.close()
    # the graph's solutions equal the plain ones, bitwise
    n_ofs = B.ofs["n"]
    xgh = xg.cpu().numpy()
    same = all(np.array_equal(xgh[n_ofs[q]:n_ofs[q + 1]], xs[q].cpu().numpy()) for q in range(count))
    st = [s.stats() for s in syms]
    sched_name = {kkt.SCHEDULE_LEVELS: "levels", kkt.SCHEDULE_QUEUE: "queue"}[best["schedule"]]
    flops = float(sum(s["flops_exact"] for s in st))
    fac_s = btm["factor"]["ms"] * 1e-3 / reps
    batch_roofline = dict(kernel="k_factor+k_update" if sched_name == "levels" else "k_factor_queue", bound="mfma",
                          unit="TFLOP/s", achieved=round(flops / fac_s / 1e12, 4), peak=PEAK_FP64_TFLOPS,
                          frac=round(flops / fac_s / 1e12 / PEAK_FP64_TFLOPS, 5),
                          launches_per_batch=btm["factor"]["launches"] / reps,
                          factor_ms_per_batch=round(1e3 * fac_s, 4))
    return dict(instances=count, sum_n=int(n_ofs[-1]), sum_nnz_l=int(sum(s["nnz_l"] for s in st)),
                flops_exact=flops, options=opts, schedule=sched_name,
                update_split=list(best.get("split", (140, 64))), small_fronts_cols=best.get("small", 0),
                roofline=batch_roofline,
                phase_ms_per_batch={p: round(btm[p]["ms"] / reps, 4) for p in btm},
                autotuned=bool(args.batch_autotune), tune_s=round(tune_s, 2), analyze_s=round(analyze_s, 2),
                tried=tuned["tried"] if tuned else None, graph_rounds=args.graph_rounds,
                batched_pairs_per_s=round(ok / tg, 2), batched_ms=round(1e3 * tg, 3),
                eager_levels_ms=round(1e3 * eager_s["levels"], 3), eager_queue_ms=round(1e3 * eager_s["queue"], 3),
                plain_pairs_per_s=round(pok / tp, 2), plain_ms=round(1e3 * tp, 3),
                speedup=round((ok / tg) / max(pok / tp, 1e-12), 2),
                plain_default_options_pairs_per_s=round(pok_d / tp_d, 2),
                speedup_vs_faster_plain=round((ok / tg) / max(pok / tp, pok_d / tp_d, 1e-12), 2),
                eta_max=float(etas.max()),
                passing=f"{ok}/{count}", batched_equals_plain_bitwise=bool(same))


def bench_stagewise(args, kkt, kktgen, torch, dev, pat, dvals, plain_ms, batch_eager_ms):
    """The stage-structured solver (block cyclic reduction over the stages, section "Future Works") on
    the paper-scale pattern and on the batched NMPC workload, beside the supernodal path's times."""
    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    def run(W, steps, get, x):
        def step(i):
            d = get(i)
            W.refactor(d["w"], d["j"], d["sx"], d["ss"])
            return W.solve(d["b"], x)
        for i in range(2):
            step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [step(i) for i in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        W.set_timing(True)
        W.read_timing()
        for i in range(steps):
            step(i)
        tm = W.read_timing()
        W.set_timing(False)
        etas = np.array([q["eta"] for inf in infos for q in inf])
        return el / steps, etas, {p: round(tm[p]["ms"] / steps, 4) for p in tm if tm[p]["launches"]}, tm

    out = {}
    s = pat.meta["stage"]
    W = kkt.Stagewise([kkt.Symbolic.from_pattern(pat)], [np.arange(0, pat.n + 1, s, dtype=np.int32)])
    x = torch.zeros(pat.n, dtype=torch.float64, device=dev)
    sec, etas, ph, tm = run(W, args.steps, lambda i: dvals[i % len(dvals)], x)
    ok = int((etas <= ETA_GATE).sum())
    out["paper"] = dict(ms_per_step=round(1e3 * sec, 4), pairs_per_s=round(ok / len(etas) / sec, 2),
                        passing=f"{ok}/{len(etas)}", eta_max=float(etas.max()), phase_ms_per_step=ph,
                        factor_launches=tm["factor"]["launches"] // args.steps,
                        supernodal_ms_per_step=round(plain_ms, 4), speedup_vs_supernodal=round(plain_ms / (1e3 * sec), 3))
    W.close()
    if args.batch > 0:
        shapes = kktgen.batch_shapes(args.batch)
        pats = [kktgen.nmpc_pattern(*sh) for sh in shapes]
        vals = [kktgen.nmpc_values(p, kktgen.rng_for(3, q, 1), 1e-6, 1e6) for q, p in enumerate(pats)]
        cat = dict(w=T(np.concatenate([v.w_vals for v in vals])), j=T(np.concatenate([v.j_vals for v in vals])),
                   sx=T(np.concatenate([v.sigma_x for v in vals])), ss=T(np.concatenate([v.sigma_s for v in vals])),
                   b=T(np.concatenate([v.b for v in vals])))
        W = kkt.Stagewise([kkt.Symbolic.from_pattern(p) for p in pats],
                          [np.arange(0, p.n + 1, p.meta["stage"], dtype=np.int32) for p in pats])
        xb = torch.zeros(sum(p.n for p in pats), dtype=torch.float64, device=dev)
        sec, etas, ph, tm = run(W, 5, lambda i: cat, xb)
        ok = int(sum(e <= ETA_GATE for e in etas[-len(pats):]))
        out["batch"] = dict(instances=len(pats), ms_per_batch=round(1e3 * sec, 4), pairs_per_s=round(ok / sec, 2),
                            passing=f"{ok}/{len(pats)}", eta_max=float(etas.max()), phase_ms_per_batch=ph,
                            factor_launches=tm["factor"]["launches"] // 5,
                            supernodal_eager_ms=batch_eager_ms,
                            speedup_vs_supernodal_eager=round(batch_eager_ms / (1e3 * sec), 3) if batch_eager_ms else None)
        W.close()
    return out


def bench_hykkt(args, kkt, kktgen, torch, dev, opts):
    """HyKKT on the paper-scale shape: refactor K_gamma = W + Sigma_x + gamma J^T J, then conjugate
    gradient on the Schur complement J K_gamma^{-1} J^T (section "Solution 2: HyKKT"), gamma = 1e7.

    Two Sigma_x ranges. The late-iteration range logU[1e-8, 1e8]: there the Schur complement's
    condition number is in the thousands and ||r|| <= 1e-10 ||c|| is out of reach, so CG stops on
    the library's bound of the saddle system's normwise backward error (eta_tol = 1e-10); a pair
    counts when the library reports success and its saddle-system eta <= 1e-10. The mid range
    logU[1e-2, 1e2]: CG to the recurrence tolerance 1e-10 (eta checked the same way)."""
    pat, _ = kktgen.paper_config()

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    gamma = 1e7
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    fac = kkt.Factor(sym)
    dx = torch.zeros(pat.n, dtype=torch.float64, device=dev)
    dy = torch.zeros(pat.m, dtype=torch.float64, device=dev)
    out = {}
    for name, (lo, hi, eta_tol) in (("late_sigma", (1e-8, 1e8, ETA_GATE)), ("mid_sigma", (1e-2, 1e2, 0.0))):
        vals = [kktgen.distillation_values(pat, kktgen.rng_for(1, 0, vs), lo, hi) for vs in range(3)]
        dv = [dict(w=T(v.w_vals), j=T(v.j_vals), sx=T(v.sigma_x), f=T(v.f), g=T(v.g)) for v in vals]

        def step(i):
            d = dv[i % len(dv)]
            fac.refactor(d["w"], d["j"], d["sx"], None, gamma)
            return fac.cg_schur(d["f"], d["g"], dx, dy, tol=1e-10, maxit=300, eta_tol=eta_tol)

        for i in range(args.warmup):
            step(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = [step(i) for i in range(args.steps)]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        fac.set_timing(True)
        fac.read_timing()
        for i in range(args.steps):
            step(i)
        tm = fac.read_timing()
        fac.set_timing(False)
        ok = sum(1 for i in infos if i["status"] == 0 and i["eta"] <= ETA_GATE)
        out[name] = dict(
            workload=f"hykkt, distillation-shaped N=2000 (n=142000, m=140000), Sigma_x~logU[{lo:g},{hi:g}], "
                     f"gamma=1e7, CG tol 1e-10" + (", eta stop 1e-10" if eta_tol else ""),
            pairs_per_s=round(ok / elapsed, 3), ms_per_pair=round(1e3 * elapsed / args.steps, 4),
            passing=f"{ok}/{args.steps}", cg_iters_mean=float(np.mean([i["iters"] for i in infos])),
            eta_stops=int(sum(i["eta_stop"] for i in infos)),
            eta_max=float(max(i["eta"] for i in infos)), rel_res_max=float(max(i["rel_res"] for i in infos)),
            phase_ms_per_pair={p: round(tm[p]["ms"] / args.steps, 4) for p in tm},
            launches_per_pair={p: round(tm[p]["launches"] / args.steps, 1) for p in tm})
        if name == "mid_sigma" and not args.no_cpu_baseline:
            # the oracle's HyKKT (sparse LDL^T of K_gamma, CG on the Schur
            # complement) on one core, one value set: context for the GPU time
            from oracle import sparse as S
            t0 = time.perf_counter()
            _, _, oinfo = S.hykkt_cg_solve(pat, vals[0], vals[0].f, vals[0].g, gamma, tol=1e-10, maxit=300)
            out[name]["cpu_oracle"] = dict(s_per_pair=round(time.perf_counter() - t0, 3), cg_iters=oinfo["iters"],
                                           status=oinfo["status"], pairs_timed=1, cores=1, kind="oracle")
    return out


def bench_large_fronts(args, kkt, kktgen, torch, dev):
    """Fronts too tall for LDS: NMPC stages 700 variables wide, nested dissection
    (its separator fronts take the large-front path in HBM), beside natural stage
    order on the same pattern (every front in LDS)."""
    pat = kktgen.nmpc_pattern(4, 700, 4)
    v = kktgen.nmpc_values(pat, kktgen.rng_for(0, 11, 0), 1e-6, 1e6)

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    d = [T(v.w_vals), T(v.j_vals), T(v.sigma_x), T(v.sigma_s)]
    b = T(v.b)
    x = torch.zeros(pat.n, dtype=torch.float64, device=dev)
    out = dict(workload="NMPC N=4 nx=700 nu=4 (n=2816, m=2800), Sigma~logU[1e-6,1e6]")
    for name, opts in (("nested_dissection", dict(ordering=kkt.ORDER_ND)), ("natural", dict(ordering=kkt.ORDER_NATURAL))):
        sym = kkt.Symbolic.from_pattern(pat, **opts)
        st = sym.stats()
        f = kkt.Factor(sym)

        def step():
            f.refactor(*d)
            return f.solve(b, x)

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = 5
        for _ in range(reps):
            info = step()
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        # per-phase kernel time from one more step under the per-launch timers (not in ms_per_pair)
        f.set_timing(True)
        f.read_timing()
        step()
        tm = f.read_timing()
        f.close()
        out[name] = dict(ms_per_pair=round(1e3 * sec, 3), eta=info["eta"],
                         large_fronts=st["large_fronts"], max_rows=st["max_rows"], levels=st["levels"],
                         flops_exact=st["flops_exact"],
                         phase_ms={k: round(tv["ms"], 4) for k, tv in tm.items() if tv["ms"]})
    return out


def bench_small(args, kkt, kktgen, torch, dev):
    """The small NMPC system (N=50, nx=8, nu=1: n=450, m=400, Sigma~logU[1e-2,1e2]) over 10 value
    sets: the plain solver one pair at a time (eager calls, and the pair replayed as a one-instance
    batch graph), and `small_batch` instances of the same pattern, each with its own value set,
    refactored and solved by one graph replay. Launch latency bounds this system; batching is what
    uses the GPU."""
    pat, _ = kktgen.small_config()
    sym = kkt.Symbolic.from_pattern(pat)
    sets = 10

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    vals = [kktgen.workload("small", 0, s)[1] for s in range(max(sets, args.small_batch))]
    dv = [dict(w=T(v.w_vals), j=T(v.j_vals), sx=T(v.sigma_x), ss=T(v.sigma_s), b=T(v.b)) for v in vals[:sets]]
    f = kkt.Factor(sym)
    x = torch.zeros(pat.n, dtype=torch.float64, device=dev)
    for d in dv:
        f.refactor(d["w"], d["j"], d["sx"], d["ss"])
        f.solve(d["b"], x)
    torch.cuda.synchronize()
    etas = []
    t0 = time.perf_counter()
    for d in dv:
        for _ in range(args.small_pairs):
            f.refactor(d["w"], d["j"], d["sx"], d["ss"])
            etas.append(f.solve(d["b"], x)["eta"])
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / len(etas)
    etas = np.array(etas)
    f.close()
    out = dict(workload="lifted-kkt plain, NMPC N=50 nx=8 nu=1 (n=450, m=400), Sigma~logU[1e-2,1e2], "
                        f"{sets} value sets x {args.small_pairs} pairs",
               plain=dict(pairs_per_s=round(1.0 / tp, 1), ms_per_pair=round(1e3 * tp, 4),
                          passing=f"{int((etas <= ETA_GATE).sum())}/{etas.size}", eta_max=float(etas.max())))

    def graph_rate(count, reps):
        B = kkt.Batch([sym] * count)
        vs = vals[:count]
        cat = {k: T(np.concatenate([getattr(v, k) for v in vs])) for k in ("w_vals", "j_vals", "sigma_x",
                                                                              "sigma_s", "b")}
        xg = torch.zeros(int(B.ofs["n"][-1]), dtype=torch.float64, device=dev)
        B.capture(cat["w_vals"], cat["j_vals"], cat["sigma_x"], cat["sigma_s"], cat["b"], xg, rounds=1)
        B.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ok = 0
        for _ in range(reps):
            infos = B.replay()
            ok += sum(i["eta"] <= ETA_GATE for i in infos)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / reps
        B.close()
        return dict(instances=count, ms_per_replay=round(1e3 * sec, 4), pairs_per_s=round(count / sec, 1),
                    passing=f"{ok}/{count * reps}")

    out["graph_one_instance"] = graph_rate(1, 200)
    if args.small_batch > 0:
        out["batched"] = graph_rate(args.small_batch, 20)
        out["batched_vs_plain"] = round(out["batched"]["pairs_per_s"] / out["plain"]["pairs_per_s"], 2)
    return out


def bench_ipm(args, kkt, kktgen, torch, dev, opts):
    """Time per interior-point iteration (section "INTERIOR-POINT METHOD") on a convex LQ-MPC QP with
    the paper-scale distillation-shaped W and J (n=142,000, m=140,000): min 1/2 x^T W x + c^T x,
    J x <= u, from x = 0, s = u, z = 1 to tol 1e-8. Each iteration is an inertia-corrected refactor with
    D_s = Z S^{-1}, the augmented solve, and the device vector kernels. The oracle's interior-point
    method (same algorithm, CPU) is timed for two iterations on the same problem."""
    from oracle import ipm as oipm
    pat, _ = kktgen.paper_config()
    v = kktgen.distillation_values(pat, kktgen.rng_for(1, 0, 0), 1e-2, 1e2)
    rng = kktgen.rng_for(100, 2, 0)
    c = rng.standard_normal(pat.n)
    u = 0.1 + rng.random(pat.m)

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    fac = kkt.Factor(kkt.Symbolic.from_pattern(pat, **opts))
    dw, dj, dc, du = T(v.w_vals), T(v.j_vals), T(c), T(u)

    def run():
        x = torch.zeros(pat.n, dtype=torch.float64, device=dev)
        s_ = du.clone()
        z = torch.ones(pat.m, dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = fac.ipm_qp(dw, dj, dc, du, x, s_, z, tol=1e-8)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    run()
    secs, info = run()
    cpu = None
    if not args.no_cpu_baseline:
        W, c2, J, u2 = oipm.qp_from_pattern(pat, v, c, u)
        t0 = time.perf_counter()
        _, _, _, oinfo = oipm.qp_ipm(W, c2, J, u2, np.zeros(pat.n), u2.copy(), np.ones(pat.m), tol=1e-8, maxit=2)
        cs = time.perf_counter() - t0
        cpu = dict(s_per_iteration=round(cs / max(1, oinfo["iterations"]), 3), iterations_timed=oinfo["iterations"],
                   cores=1, kind="oracle")
    its = max(1, info["iterations"])
    return dict(workload="convex QP, distillation-shaped N=2000 W and J (n=142000, m=140000), J x <= u, tol 1e-8",
                status=info["status"], iterations=info["iterations"], ms_total=round(1e3 * secs, 3),
                ms_per_iteration=round(1e3 * secs / its, 3), err=info["err"], max_delta=info["max_delta"],
                cpu_oracle=cpu)


def bench_served(args, kkt, kktgen, torch, dev):
    """Poisson stream over 16 resident patterns: continuous batching vs plain FIFO."""
    shapes = kktgen.serving_shapes(16)
    pats = [kktgen.nmpc_pattern(*sh) for sh in shapes]
    syms = [kkt.Symbolic.from_pattern(p) for p in pats]
    nvs = 3

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    pool = []
    for p, pat in enumerate(pats):
        vs = [kktgen.nmpc_values(pat, kktgen.rng_for(4, p, 1 + r), 1e-6, 1e6) for r in range(nvs)]
        pool.append([[T(v.w_vals), T(v.j_vals), T(v.sigma_x), T(v.sigma_s), T(v.b)] for v in vs])
    # plain capacity on this mix: mean service time of one request alone
    plain = kkt.Server(hbm_budget=16 << 30, max_wave=1, workers=1)
    pid = [plain.register(s) for s in syms]
    xbuf = [torch.zeros(p.n, dtype=torch.float64, device=dev) for p in pats]
    for p in range(16):
        plain.wait(plain.submit(pid[p], *pool[p][0], xbuf[p]))
    plain.reset_stats()
    for rep in range(2):
        for p in range(16):
            plain.wait(plain.submit(pid[p], *pool[p][rep % nvs], xbuf[p]))
    svc = plain.stats()["mean_service_s"]
    capacity = 1.0 / svc
    nreq = args.serve_requests
    warm = nreq // 20

    def run(server, pids, times, which):
        outs = [[torch.zeros(p.n, dtype=torch.float64, device=dev) for _ in range(8)] for p in pats]
        tickets = []
        t0 = time.perf_counter()
        for k in range(nreq):
            delay = t0 + times[k] - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            p = int(which[k])
            if k == warm:
                server.reset_stats()
            tickets.append(server.submit(pids[p], *pool[p][k % nvs], outs[p][k % 8]))
        res = [server.wait(t) for t in tickets]
        st = server.stats()
        bad = sum(r["status"] != 0 or r["eta"] > ETA_GATE for r in res)
        return st, bad

    def pick(st):
        return {k: (round(st[k] * 1e3, 3) if k.endswith("_s") else round(st[k], 3)) for k in
                ("p50_s", "p99_s", "mean_queue_s", "mean_service_s", "throughput", "mean_wave")}

    cb = kkt.Server(hbm_budget=16 << 30, max_wave=64, workers=args.serve_workers)
    cid = [cb.register(s) for s in syms]
    by_rho = []
    for rho in [float(r) for r in str(args.serve_rho).split(",") if r]:
        rate = rho * capacity
        times, which = kktgen.poisson_arrivals(rate, nreq, 16)
        plain.reset_stats()
        pst, pbad = run(plain, pid, times, which)
        cst, cbad = run(cb, cid, times, which)
        by_rho.append(dict(rho=rho, rate_per_s=round(rate, 2), continuous_batching=pick(cst), plain_fifo=pick(pst),
                           failed=int(cbad), plain_failed=int(pbad)))
        print(f"served rho={rho}: p99 {by_rho[-1]['continuous_batching']['p99_s']} ms "
              f"(plain {by_rho[-1]['plain_fifo']['p99_s']} ms)", file=sys.stderr, flush=True)
    plain.close()
    cb.close()
    return dict(patterns=16, n_range=[min(p.n for p in pats), max(p.n for p in pats)], requests_per_rate=nreq,
                warmup_discarded=warm, plain_capacity_per_s=round(capacity, 2), workers=args.serve_workers,
                units="latencies in ms, throughput in requests/s", by_rho=by_rho)


# kernels launched under each timed phase
PHASE_KERNELS = {"factor": "k_factor+k_update", "fwd": "k_fwd", "bwd": "k_bwd", "assemble": "k_assemble",
                 "residual": "k_residual"}


def measured_traffic(phase, args, opts, launches_per_step):
    """HBM bytes per launch of a phase from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a plain copy's reading): the
    phase's bytes per refactor there over this run's launches per step, or
    None when the kernels changed since the counters were taken or another
    configuration (workload, schedule, symbolic options) is benchmarked."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    src = os.path.join(ROOT, "paper_2403_15913_amd", "csrc", "kernels.hip")
    if args.workload != "paper" or args.schedule != "levels":
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
        with open(src, "rb") as fh:
            sha = hashlib.sha256(fh.read()).hexdigest()
    except OSError:
        return None
    if rec.get("kernels_sha256") != sha or rec.get("options") != {k: int(v) for k, v in opts.items()}:
        return None
    ph = rec.get("phases", {}).get(phase)
    if ph:
        if "bytes_per_refactor" in ph:
            return round(ph["bytes_per_refactor"] / max(1.0, launches_per_step))
        return round(ph["bytes_per_launch"])
    k = rec.get("per_launch", {}).get(PHASE_KERNELS.get(phase, ""))
    return round(k["fetch_bytes"] + k["write_bytes"]) if k else None


_CPU_WORK = None  # (pattern, value sets) inherited by the forked oracle workers


def _oracle_pairs(idx):
    """Oracle refactor+solve pairs (value sets idx, in turn); returns how many pass the gate."""
    from oracle import sparse as S
    pat, vals = _CPU_WORK
    ok = 0
    for i in idx:
        v = vals[i % len(vals)]
        _, oinfo = S.lifted_solve(pat, v, v.b)
        ok += int(oinfo["spd"] and oinfo["eta"] <= ETA_GATE)
    return ok


def cpu_baseline(args, pat, vals):
    """The FP64 oracle (scipy assembly + C up-looking sparse LDL^T in stage order + Richardson
    refinement) on the host: one process per core over the cores this process may run on (at most
    16, the host share of one GPU), and a single core for reference."""
    import concurrent.futures as cf
    import multiprocessing as mp
    global _CPU_WORK
    from oracle.build import build_oracle
    build_oracle(force=False)
    _CPU_WORK = (pat, vals)
    affinity = len(os.sched_getaffinity(0))
    cores = max(1, min(affinity, 16))
    ns1 = max(1, args.cpu_sample // 2)
    t0 = time.perf_counter()
    ok1 = _oracle_pairs(range(ns1))
    s1 = time.perf_counter() - t0
    per = max(2, args.cpu_sample // (2 * cores))
    nsa = per * cores
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("fork")) as ex:
        list(ex.map(_oracle_pairs, [[0]] * cores))  # workers started and warm
        t0 = time.perf_counter()
        oka = sum(ex.map(_oracle_pairs, [range(w * per, (w + 1) * per) for w in range(cores)]))
        sa = time.perf_counter() - t0
    return dict(value=round(oka / sa, 4), unit="refactor+solves/s", cores=cores, kind="oracle",
                sample=f"{nsa} refactor+solve pairs of the same workload ({per} per process, value sets in turn) "
                       f"on {cores} processes, one per core (sched_getaffinity: {affinity} cores): scipy assembly "
                       f"+ C up-looking sparse LDL^T in stage order + Richardson refinement",
                seconds=round(sa, 3), affinity_cores=affinity,
                single_core=dict(value=round(ok1 / s1, 4), cores=1, pairs=ns1, seconds=round(s1, 3)))


def algorithmic_work(stats, pat, n_steps, sweeps_per_step, residuals_per_step, nnz_k_full):
    """Minimal bytes / flops of each phase over the timed steps."""
    n, m = pat.n, pat.m
    nl = stats["nnz_l_exact"]
    return {
        "assemble": dict(bound="hbm", unit="GB/s",
                         work=n_steps * 8.0 * (pat.nnz_w + pat.nnz_j + n + m + stats["nnz_k"])),
        "factor": dict(bound="mfma", unit="TFLOP/s", work=n_steps * stats["flops_exact"]),
        "fwd": dict(bound="hbm", unit="GB/s", work=sweeps_per_step * n_steps * (8.0 * nl + 16.0 * n)),
        "bwd": dict(bound="hbm", unit="GB/s", work=sweeps_per_step * n_steps * (8.0 * nl + 16.0 * n)),
        "residual": dict(bound="hbm", unit="GB/s", work=residuals_per_step * n_steps * (12.0 * nnz_k_full + 24.0 * n)),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library runs each solve on a single MI355X "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import kktgen
    from paper_2403_15913_amd import kkt

    dev = torch.device("cuda:0")
    if args.copy_probe_mib > 0:
        # reads and writes exactly copy_probe_mib MiB each: the scale of FETCH_SIZE / WRITE_SIZE
        n = args.copy_probe_mib << 17
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_mib": args.copy_probe_mib, "bytes_each_way": 8 * n}), flush=True)
        return
    gen = {"paper": (1, kktgen.paper_config, kktgen.distillation_values),
           "small": (0, kktgen.small_config, kktgen.nmpc_values)}[args.workload]
    cfg_idx, cfg_fn, val_fn = gen
    pat, (slo, shi) = cfg_fn()
    vals = [val_fn(pat, kktgen.rng_for(cfg_idx, 0, vs), slo, shi) for vs in range(args.value_sets)]
    # the oracle on the host cores, before anything touches the GPU (its worker processes are forked)
    cpu = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        cpu = cpu_baseline(args, pat, vals)
    kkt.lib()

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    dvals = [dict(w=T(v.w_vals), j=T(v.j_vals), sx=T(v.sigma_x), ss=T(v.sigma_s), b=T(v.b)) for v in vals]
    x = torch.zeros(pat.n, dtype=torch.float64, device=dev)

    tuned = None
    opts = dict(ordering=args.ordering, nd_leaf=args.nd_leaf, max_super=args.max_super)
    split = (140, 64)  # the library's default launch shape of the update matrices
    small = 0  # the library's default: every front by eight-wave workgroups (column threshold 0)
    if args.autotune and not args.ordering and not args.nd_leaf:
        from paper_2403_15913_amd import autotune
        t0 = time.perf_counter()
        tried = []
        best = autotune.tune_pattern(pat, vals[0], reps=3, table_path=None, log=tried.append,
                                     schedules=(kkt.SCHEDULE_LEVELS, kkt.SCHEDULE_QUEUE))
        opts = {k: best[k] for k in ("ordering", "nd_leaf", "max_super")}
        if args.schedule_given is None:
            args.schedule = "queue" if best["schedule"] == kkt.SCHEDULE_QUEUE else "levels"
        split = tuple(best["split"])
        small = int(best.get("small", 0))
        tuned = dict(seconds=round(time.perf_counter() - t0, 2), tried=tried)
    t0 = time.perf_counter()
    sym = kkt.Symbolic.from_pattern(pat, **opts)
    analyze_s = time.perf_counter() - t0
    stats = sym.stats()
    fac = kkt.Factor(sym)
    fac.set_schedule(kkt.SCHEDULE_QUEUE if args.schedule == "queue" else kkt.SCHEDULE_LEVELS)
    fac.set_update_split(*split)
    fac.set_small_fronts(small)

    def step(i):
        d = dvals[i % len(dvals)]
        fac.refactor(d["w"], d["j"], d["sx"], d["ss"])
        return fac.solve(d["b"], x)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()

    infos = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(step(i))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    etas = np.array([inf["eta"] for inf in infos])
    passing = int((etas <= ETA_GATE).sum())
    value = passing / elapsed
    ms_per_step = 1e3 * elapsed / args.steps

    # live per-kernel timing over a second pass of the same steps
    fac.set_timing(True)
    fac.read_timing()
    torch.cuda.synchronize()
    tinfos = [step(i) for i in range(args.steps)]
    tm = fac.read_timing()
    fac.set_timing(False)
    iters = np.array([inf["iters"] for inf in tinfos])
    sweeps_per_step = 1.0 + iters.mean()
    residuals_per_step = tm["residual"]["launches"] / args.steps
    nnz_k_full = 2 * stats["nnz_k"] - pat.n
    work = algorithmic_work(stats, pat, args.steps, sweeps_per_step, residuals_per_step, nnz_k_full)
    phase_ms = {p: tm[p]["ms"] / args.steps for p in tm}
    if tm["bwd"]["launches"] == 0:
        # queue schedule: one launch runs both sweeps (counted under fwd)
        work["fwd"]["work"] += work["bwd"]["work"]
        del work["bwd"]
    dom = max(work, key=lambda p: tm[p]["ms"])
    wd = work[dom]
    secs = tm[dom]["ms"] * 1e-3
    if wd["unit"] == "TFLOP/s":
        achieved, peak = wd["work"] / secs / 1e12, PEAK_FP64_TFLOPS
    else:
        achieved, peak = wd["work"] / secs / 1e9, PEAK_HBM_GBS
    kernel = PHASE_KERNELS.get(dom, f"k_{dom}")
    if args.schedule == "queue":
        kernel = {"factor": "k_factor_queue", "fwd": "k_sweeps_queue"}.get(dom, kernel)
    roofline = dict(bound=wd["bound"], achieved=round(achieved, 4), peak=peak, unit=wd["unit"],
                    frac=round(achieved / peak, 5),
                    traffic=measured_traffic(dom, args, opts, tm[dom]["launches"] / args.steps), traffic_unit="bytes/launch",
                    kernel=kernel, launches_per_step=tm[dom]["launches"] / args.steps,
                    avg_launch_us=1e3 * tm[dom]["ms"] / max(1, tm[dom]["launches"]))
    if dom == "factor":
        # the binding roof min(P_mfma, AI * BW), AI = exact flops over the minimal bytes (L written once
        # and read once: 16 nnz(L))
        ai = stats["flops_exact"] / (16.0 * stats["nnz_l_exact"])
        binding = min(PEAK_FP64_TFLOPS, ai * PEAK_HBM_GBS / 1e3)
        roofline.update(arithmetic_intensity=round(ai, 3), binding_roof=round(binding, 3),
                        frac_of_binding_roof=round(achieved / binding, 5))

    hykkt = bench_hykkt(args, kkt, kktgen, torch, dev, opts) if args.hykkt and args.workload == "paper" else None
    ipm_leg = bench_ipm(args, kkt, kktgen, torch, dev, opts) if args.ipm and args.workload == "paper" else None
    batched = bench_batched(args, kkt, kktgen, torch, dev) if args.batch > 0 else None
    served = bench_served(args, kkt, kktgen, torch, dev) if args.serve_requests > 0 else None
    large = bench_large_fronts(args, kkt, kktgen, torch, dev) if args.large_fronts else None
    small_leg = bench_small(args, kkt, kktgen, torch, dev) if args.small else None
    stagewise = None
    if args.stagewise and args.workload == "paper":
        stagewise = bench_stagewise(args, kkt, kktgen, torch, dev, pat, dvals, ms_per_step,
                                    batched["eager_levels_ms"] if batched else None)

    out = {
        "metric": "KKT refactor+solves/sec at residual <=1e-10 (batched vs plain); served p50/p99",
        "value": round(value, 3),
        "unit": "refactor+solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": ("lifted-kkt plain, distillation-shaped N=2000 (n=142000, m=140000), "
                                "Sigma~logU[1e-8,1e8], 10 value sets") if args.workload == "paper"
                   else "lifted-kkt plain, NMPC N=50 nx=8 nu=1 (n=450, m=400)",
                   "mode": "plain", "options": opts, "autotuned": tuned is not None,
                   "schedule": args.schedule, "update_split": list(split), "small_fronts_cols": small},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "pairs_passing_eta": f"{passing}/{args.steps}",
            "eta_max": float(etas.max()),
            "refine_iters_mean": float(iters.mean()),
            "analyze_s": round(analyze_s, 4),
            "autotune": tuned,
            "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
            "symbolic": {k: stats[k] for k in ("nsuper", "levels", "max_rows", "max_cols", "nnz_k", "nnz_l",
                                               "nnz_l_exact", "flops", "flops_exact")},
            "hykkt": hykkt,
            "ipm": ipm_leg,
            "batched": batched,
            "served": served,
            "stagewise": stagewise,
            "large_fronts": large,
            "small": small_leg,
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
