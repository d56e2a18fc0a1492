"""Writes ex3_counts.json: iteration counts of the oracle's TBAS(10),
tGMRES(10) and tFOM(10) on the experiment family of section 6 (the
convection-diffusion slices of workloads.ex3 at n = 1000, s = 3, p = 2, with
mu = 1e-3: the paper does not give mu, so Table 1 itself is not reproduced;
these counts pin the qualitative ordering the table reports, TBAS ahead of
tGMRES ahead of tFOM).  Calls only the oracle and the input generator.

The restart count of TBAS(10) on this case is decided at the rounding
level: its residual first grows (to about 2e3 by cycle 100) and then falls
along a path that rounding changes, so the oracle's own count moves by
tens of percent when C is perturbed by one unit in the last place, while
the first 100 cycles agree to four digits.  The script records the
oracle's counts for five such perturbations (C times 1 + 1e-15 xi, xi
standard normal from numpy's default_rng(seed), seeds 1..5) and the
unperturbed run's residual estimates of the first 100 cycles, which are
what the GPU test holds its own to.

    python tests/golden/make_ex3_counts.py      (about five minutes, 5 processes)
"""

import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import krylov  # noqa: E402
from paper_2405_09233_amd import workloads  # noqa: E402

N, S, P, MU, M, TOL = 1000, 3, 2, 1e-3, 10, 1e-6
GMRES_CYCLES, FOM_CYCLES = 100, 20
PERTURB_EPS, PERTURB_SEEDS = 1e-15, (1, 2, 3, 4, 5)
HIST_CYCLES = 100


def _tbas_cycles(seed):
    """TBAS(10) restart cycles with C perturbed at the rounding level
    (seed None: unperturbed)."""
    import numpy as np
    A, B, C = workloads.ex3(N, S, P, mu=MU)
    if seed is not None:
        xi = np.random.default_rng(seed).standard_normal(C.shape)
        C = C * (1.0 + PERTURB_EPS * xi)
    _, it = krylov.tbas(A, B, C, m=M, tol=TOL, max_cycles=600)
    return it


def main():
    A, B, C = workloads.ex3(N, S, P, mu=MU)
    with ProcessPoolExecutor(max_workers=len(PERTURB_SEEDS)) as pool:
        perturbed = list(pool.map(_tbas_cycles, PERTURB_SEEDS))
    _, it = krylov.tbas(A, B, C, m=M, tol=TOL, max_cycles=600)
    _, ig = krylov.tgmres(A, B, C, m=M, tol=TOL, max_cycles=GMRES_CYCLES)
    try:
        _, iff = krylov.tfom(A, B, C, m=M, tol=TOL, max_cycles=FOM_CYCLES)
        fom = {"cycles": iff["cycles"], "relres_true": iff["relres_true"],
               "converged": iff["converged"], "fom_fallback": iff["fom_fallback"]}
    except krylov.SingularProjected as e:
        fom = {"singular": str(e)}
    out = {
        "source": "oracle (tests/golden/make_ex3_counts.py); workload: workloads.ex3(%d, %d, %d, "
                  "mu=%g), seed 0; restart length %d, tol %g" % (N, S, P, MU, M, TOL),
        "cite": "section 6, Table 1 (qualitative ordering only: mu and the rand stream of the "
                "experiment are not given)",
        "tbas": {"cycles": it["cycles"], "converged": it["converged"],
                 "relres_true": it["relres_true"],
                 "est_hist_first": [float(x) for x in it["est_hist"][:HIST_CYCLES]],
                 "perturbed": {"eps": PERTURB_EPS, "seeds": list(PERTURB_SEEDS),
                               "cycles": [q["cycles"] for q in perturbed],
                               "converged": [bool(q["converged"]) for q in perturbed]}},
        "tgmres": {"cycles": ig["cycles"], "converged": ig["converged"],
                   "relres_true": ig["relres_true"]},
        "tfom": fom,
    }
    with open(os.path.join(HERE, "ex3_counts.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
