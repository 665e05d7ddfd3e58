"""Oracle-only reference runs of the propagator workloads.

Solves Dw psi = eta with the oracle's full-lattice FP64 CG (no even-odd
preconditioning) for the first point source (x = 0, spin 0, colour 0) of a
workload, to a true residual of 1e-10, links exp(i 0.2 H), periodic space and
antiperiodic time, csw = 1.9:
  c2: 16^3x32, kappa 0.1345, link seed 2  -> c2_reference.json
  c3: 32^3x64, kappa 0.135,  link seed 3  -> c3_reference.json
The number of CG iterations it needs is written to the json file; the
benchmark's CPU-baseline leg times a bounded number of oracle iterations and
scales by this count.  Calls nothing but the oracle and the seeded input
generator.

    python oracle/reference_run.py [c2|c3]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as orc  # noqa: E402
from paper_2503_16994_amd import inputs  # noqa: E402

WORKLOADS = {"c2": ((16, 16, 16, 32), 0.1345, 2), "c3": ((32, 32, 32, 64), 0.135, 3)}
CSW, EPS, TOL = 1.9, 0.2, 1e-10
THETA = (1, 1, 1, -1)


def main(name="c2"):
    L, KAPPA, SEED = WORKLOADS[name]
    U = inputs.gauge_field(L, EPS, seed=SEED)
    A = orc.clover_matrix(L, orc.PERIODIC, U, orc.m0_from_kappa(KAPPA), CSW)
    eta = inputs.point_source(L, (0, 0, 0, 0), 0, 0)
    t0 = time.time()
    psi, rho, iters, ok = orc.cg(L, orc.PERIODIC, THETA, U, A, eta, TOL)
    dt = time.time() - t0
    out = {"lattice": L, "kappa": KAPPA, "csw": CSW, "eps": EPS, "seed": SEED, "tol": TOL,
           "source": "point (0,0,0,0) spin 0 colour 0", "solver": "oracle full-lattice FP64 CG",
           "iterations": iters, "true_residual": rho, "converged": ok,
           "seconds": dt, "threads": orc.num_threads()}
    with open(os.path.join(HERE, f"{name}_reference.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c2")
