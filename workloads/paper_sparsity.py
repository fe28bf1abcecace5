"""Scale of ws3's lengthscales that gives its lattice the paper's sparsity.

The paper's Houseelectric lattice (n = 2,049,280, d = 11) holds 1,000,190
lattice points, about 4.1% of its n (d+1) simplex vertices (Section 5, the
lattice-size table). ws3 with its own lengthscales has about 0.65%. This
script bisects a common factor c (on a log scale) so that the oracle's
lattice of ws3's points with lengthscales c * l has the same ratio
m / (n (d+1)), and writes c to ws3p_scale.json beside it. It calls only the
oracle (CPU, a few minutes):

    python -m workloads.paper_sparsity
"""
from __future__ import annotations

import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TARGET = 1_000_190 / (2_049_280 * 12)  # the paper's m / (n (d+1)) for Houseelectric
OUT = os.path.join(HERE, "ws3p_scale.json")


def main(iters: int = 10) -> float:
    sys.path.insert(0, os.path.dirname(HERE))
    import oracle
    import workloads
    w = workloads.ws3()
    L = w.X.shape[0] * (w.X.shape[1] + 1)

    def ratio(c):
        lat = oracle.Lattice(w.X, w.lengthscales * c)
        r = lat.m / L
        print(f"c = {c:.6f}: m = {lat.m}, m/L = {r:.5f}", flush=True)
        return r

    lo, hi = math.log(0.5), math.log(1.0)  # ratio(e^lo) > TARGET > ratio(e^hi)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if ratio(math.exp(mid)) > TARGET:
            lo = mid
        else:
            hi = mid
    c = math.exp(0.5 * (lo + hi))
    r = ratio(c)
    with open(OUT, "w") as f:
        json.dump({"scale": c, "m_over_L": r, "target": TARGET,
                   "note": "written by workloads/paper_sparsity.py from the oracle's lattice of ws3"}, f,
                  indent=1)
        f.write("\n")
    return c


if __name__ == "__main__":
    print(main())
