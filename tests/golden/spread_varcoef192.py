"""Writes spread_varcoef192.json: how far the oracle's own folded pipelined
Jacobi-CG iterate on the 7.08M-cell lognormal workload moves, at the 1,250
iterations the solve to 1e-8 takes, when only the order of its floating-point
sums changes (the same system with its cells randomly renumbered).  The GPU
parity test at full size compares its difference from the oracle with this.
Calls only the oracle and the seeded input generators:

    python tests/golden/spread_varcoef192.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fvcases as fc  # noqa: E402
import oracle  # noqa: E402
from fvcases.mesh import renumber  # noqa: E402


def renumbered(case, seed):
    new_index = np.random.default_rng(seed).permutation(case.n).astype(np.int64)
    o, nb, up, lo, _ = renumber(case.n, case.owner.astype(np.int64), case.neighbour.astype(np.int64), case.upper,
                                case.lower, new_index)
    d = np.empty_like(case.diag)
    d[new_index] = case.diag
    b = np.empty_like(case.b)
    b[new_index] = case.b
    return fc.Case(case.name, case.shape, case.n, o.astype(np.int32), nb.astype(np.int32), d, up, lo, b), new_index


def main(iters=1250, seeds=(0, 1)):
    oracle.build(force=False)
    case = fc.make("varcoef192")
    t0 = time.time()
    _, s_tol = oracle.pipecg(case, case.b, tol=1e-8, maxit=50000, folded=True, omp=True)
    xo, _ = oracle.pipecg(case, case.b, tol=0.0, maxit=iters, folded=True, omp=True)
    xc, _ = oracle.cg(case, case.b, tol=0.0, maxit=iters, omp=True)
    out = {"workload": "varcoef192", "method": "pipecg folded, Jacobi", "iters": iters,
           "oracle_iters_to_1e-8": s_tol["iters"],
           "cg_vs_pipecg_at_equal_count": float(np.linalg.norm(xc - xo) / np.linalg.norm(xo)), "renumbered": []}
    for seed in seeds:
        pc, ni = renumbered(case, seed)
        _, sp = oracle.pipecg(pc, pc.b, tol=1e-8, maxit=50000, folded=True, omp=True)
        xp, _ = oracle.pipecg(pc, pc.b, tol=0.0, maxit=iters, folded=True, omp=True)
        out["renumbered"].append({"seed": seed, "iters_to_1e-8": sp["iters"],
                                  "rel_diff": float(np.linalg.norm(xp[ni] - xo) / np.linalg.norm(xo))})
        print(out, flush=True)
    out["max_rel_diff"] = max(r["rel_diff"] for r in out["renumbered"])
    out["max_iter_change"] = max(abs(r["iters_to_1e-8"] - s_tol["iters"]) for r in out["renumbered"])
    out["seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, "spread_varcoef192.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
