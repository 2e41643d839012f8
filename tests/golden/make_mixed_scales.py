"""Write mixed_scales.json: for the mixed-precision workload L(s) = D + s N0
(D and N0 the diagonal and strict lower triangle of the standard real draw,
seed 3), the scale s at which the estimated condition number
kappa_inf(L) ~ ||L||_inf * max_j ||inv(L) z_j||_inf  (z_j random +-1 vectors,
a lower bound on kappa_inf) reaches each target, found by bisection on
log(s).  Uses only the oracle's solver.  Run from the repository root:
    python tests/golden/make_mixed_scales.py
"""
import json
import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import workloads as W  # noqa: E402

TARGETS = [1e3, 1e4, 1e5, 1e6]


def kappa_estimate(L0, off_mask_scale, s, Z):
    L = L0.copy(order="F")
    L[off_mask_scale] *= s
    X = oracle.solve(L, Z, 1.0)
    Lt = np.nan_to_num(L, nan=0.0)
    norm_l = np.max(np.abs(np.tril(Lt)).sum(axis=1))
    return float(norm_l * np.max(np.abs(X)))


def scales_for(m):
    L0 = W.lower_matrix(np.random.default_rng(3), m)
    mask = np.tril(np.ones((m, m), dtype=bool), -1)
    Z = np.asfortranarray(np.random.default_rng(33).choice([-1.0, 1.0], size=(m, 4)))
    out = {}
    lo, hi = 1.0, 2048.0
    for target in TARGETS:
        a, b = math.log(lo), math.log(hi)
        for _ in range(24):
            mid = 0.5 * (a + b)
            if kappa_estimate(L0, mask, math.exp(mid), Z) < target:
                a = mid
            else:
                b = mid
        s = math.exp(0.5 * (a + b))
        out[f"{target:.0e}"] = {"scale": s, "kappa_estimate": kappa_estimate(L0, mask, s, Z)}
        lo = s
        print(m, target, out[f"{target:.0e}"], flush=True)
    return out


if __name__ == "__main__":
    res = {"recipe": __doc__.strip().splitlines()[0:6], "seed": 3}
    for m in (1024, 8192):
        res[str(m)] = scales_for(m)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "mixed_scales.json"), "w") as f:
        json.dump(res, f, indent=1)
