"""Writes ex3_counts.json: iteration counts of the oracle's TBAS(10),
tGMRES(10) and tFOM(10) on the experiment family of section 6 (the
convection-diffusion slices of workloads.ex3 at n = 1000, s = 3, p = 2, with
mu = 1e-3: the paper does not give mu, so Table 1 itself is not reproduced;
these counts pin the qualitative ordering the table reports, TBAS ahead of
tGMRES ahead of tFOM).  Calls only the oracle and the input generator.

    python tests/golden/make_ex3_counts.py      (about three minutes)
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import krylov  # noqa: E402
from paper_2405_09233_amd import workloads  # noqa: E402

N, S, P, MU, M, TOL = 1000, 3, 2, 1e-3, 10, 1e-6
GMRES_CYCLES, FOM_CYCLES = 100, 20


def main():
    A, B, C = workloads.ex3(N, S, P, mu=MU)
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
                 "relres_true": it["relres_true"]},
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
