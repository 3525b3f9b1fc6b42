"""Write the stored expected values under tests/golden/ from the oracle alone.

Run: python tests/golden/make_golden.py

small_pattern_stats.json -- pattern statistics of the small NMPC workload
(N=50, nx=8, nu=1) under the natural (stage-major) ordering, from the
brute-force boolean elimination in oracle/symbolic.py. They depend on the
sparsity pattern only: nnz(J), nnz of the lower triangle of
K = W + Sigma_x + J^T Sigma_s J, nnz(L) including the diagonal, and the sum of
squared column counts (the factor's multiply-add count up to lower-order terms).
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import kktgen  # noqa: E402
from oracle import symbolic  # noqa: E402


def main():
    pat, _ = kktgen.small_config()
    K = symbolic.k_pattern(pat)
    st = symbolic.stats(symbolic.cholesky_structure(K))
    out = dict(workload="NMPC N=50 nx=8 nu=1, natural stage-major ordering",
               n=pat.n, m=pat.m, nnz_j=pat.nnz_j, nnz_k_lower=int((K.nnz + pat.n) // 2),
               nnz_l=st["nnz_l"], sum_c2=st["sum_c2"])
    with open(os.path.join(HERE, "small_pattern_stats.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(out)


if __name__ == "__main__":
    main()
