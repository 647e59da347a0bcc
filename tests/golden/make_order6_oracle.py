"""Writes order6_oracle.json: the oracle on the Section 4 order-6 experiment (Krylov
TT-vectors of the Dirichlet Laplacian: d = 6, n = 15, m = 35, delta = 1e-5, FP64) for
each scheme -- the loss of orthogonality ||I_k - Q_k^T Q_k||_2 for k = 1..m, the ranks of
every q_i before and after its last rounding, and the R factor's diagonal.  Calls only
oracle/; each scheme's entry is written as soon as it is done (hours of CPU in all).

Usage: python tests/golden/make_order6_oracle.py [scheme ...]
"""
import json
import os
import sys
import time

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "..", ".."))
import numpy as np  # noqa: E402

import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "order6_oracle.json")
NS, M, DELTA = [15] * 6, 35, 1e-5


def main(schemes):
    data = {"workload": "Section 4 order-6 experiment: d=6, n=15, m=35 Krylov TT-vectors "
                        "(ones, -Delta_d, rank-one rounding, normalisation), delta=1e-5, FP64",
            "schemes": {}}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    A = oracle.krylov_inputs(NS, M)
    for sch in schemes:
        t0 = time.time()
        try:
            res = oracle.orthogonalize(sch, A, DELTA)
        except (oracle.GramBreakdown, oracle.HouseholderBreakdown) as e:
            data["schemes"][sch] = {"status": type(e).__name__, "seconds": round(time.time() - t0, 1)}
        else:
            data["schemes"][sch] = {
                "loo": [float(v) for v in oracle.loo_curve(res.Q)],
                "pre_ranks": [list(map(int, r)) for r in res.pre_ranks],
                "post_ranks": [list(map(int, r)) for r in res.post_ranks],
                "q_ranks": [list(map(int, oracle.tt_ranks(q))) for q in res.Q],
                "r_diag": [float(v) for v in np.diag(res.R)],
                "rounds": int(res.rounds),
                "seconds": round(time.time() - t0, 1)}
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1)
        print(sch, data["schemes"][sch].get("seconds"), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["cgs", "mgs", "cgs2", "mgs2", "gram", "householder"])
