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
    ap.add_argument("--cpu-sample", type=int, default=4, help="oracle refactor+solve pairs timed for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--ordering", type=int, default=0)
    ap.add_argument("--nd-leaf", type=int, default=0)
    return ap.parse_args()


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
              "(multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    import kktgen
    from paper_2403_15913_amd import kkt

    dev = torch.device("cuda:0")
    kkt.lib()
    gen = {"paper": (1, kktgen.paper_config, kktgen.distillation_values),
           "small": (0, kktgen.small_config, kktgen.nmpc_values)}[args.workload]
    cfg_idx, cfg_fn, val_fn = gen
    pat, (slo, shi) = cfg_fn()
    vals = [val_fn(pat, kktgen.rng_for(cfg_idx, 0, vs), slo, shi) for vs in range(args.value_sets)]

    def T(a):
        return torch.tensor(np.asarray(a), dtype=torch.float64, device=dev)

    dvals = [dict(w=T(v.w_vals), j=T(v.j_vals), sx=T(v.sigma_x), ss=T(v.sigma_s), b=T(v.b)) for v in vals]
    x = torch.zeros(pat.n, dtype=torch.float64, device=dev)

    t0 = time.perf_counter()
    sym = kkt.Symbolic.from_pattern(pat, ordering=args.ordering, nd_leaf=args.nd_leaf)
    analyze_s = time.perf_counter() - t0
    stats = sym.stats()
    fac = kkt.Factor(sym)

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
    dom = max(work, key=lambda p: tm[p]["ms"])
    wd = work[dom]
    secs = tm[dom]["ms"] * 1e-3
    if wd["unit"] == "TFLOP/s":
        achieved, peak = wd["work"] / secs / 1e12, PEAK_FP64_TFLOPS
    else:
        achieved, peak = wd["work"] / secs / 1e9, PEAK_HBM_GBS
    roofline = dict(bound=wd["bound"], achieved=round(achieved, 4), peak=peak, unit=wd["unit"],
                    frac=round(achieved / peak, 5), traffic=None, kernel=f"k_{dom}",
                    launches_per_step=tm[dom]["launches"] / args.steps,
                    avg_launch_us=1e3 * tm[dom]["ms"] / max(1, tm[dom]["launches"]))

    cpu = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        from oracle import sparse as S
        from oracle.build import build_oracle
        build_oracle(force=False)
        ns = min(args.cpu_sample, len(vals))
        t0 = time.perf_counter()
        ok = 0
        for v in vals[:ns]:
            xo, oinfo = S.lifted_solve(pat, v, v.b)
            ok += int(oinfo["spd"] and oinfo["eta"] <= ETA_GATE)
        cs = time.perf_counter() - t0
        cpu = dict(value=round(ok / cs, 4), unit="refactor+solves/s", cores=1, kind="oracle",
                   sample=f"{ns} refactor+solve pairs (value sets 0..{ns - 1}) of the same workload: "
                          f"scipy assembly + C up-looking sparse LDL^T in stage order + Richardson refinement, "
                          f"single thread", seconds=round(cs, 3))

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
                   "mode": "plain", "ordering": args.ordering, "nd_leaf": args.nd_leaf},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {
            "pairs_passing_eta": f"{passing}/{args.steps}",
            "eta_max": float(etas.max()),
            "refine_iters_mean": float(iters.mean()),
            "analyze_s": round(analyze_s, 4),
            "phase_ms_per_step": {k: round(v, 4) for k, v in phase_ms.items()},
            "symbolic": {k: stats[k] for k in ("nsuper", "levels", "max_rows", "max_cols", "nnz_k", "nnz_l",
                                               "nnz_l_exact", "flops", "flops_exact")},
        },
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
