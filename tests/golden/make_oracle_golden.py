"""Write the oracle's reference solutions used by the GPU parity tests.

Calls only the oracle and the seeded input generators.  Each workload is
solved by the oracle's interior-point continuation (sparse direct Newton
solves) with the last mu solved to |F| <= 1e-10, so the stored solution is
the unique solution of the final relaxed system up to that residual.

    python tests/golden/make_oracle_golden.py [name ...]

Workloads:
  cfg2_64x64_K32: 64 x 64 right-triangle grid, K = 32, 3-Gaussian mixtures
      (seeded), mu = 0.2^l down to 5.12e-7;
  bg_32x32_K16: 32 x 32 grid, K = 16, 5-Gaussian mixtures plus a 1e-3
      background (the 256^2 benchmark's recipe at a size the oracle solves
      in seconds).
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import otinputs  # noqa: E402
from oracle.ipm import Problem, solve_ipm  # noqa: E402
from oracle.mesh import structured_mesh  # noqa: E402

WORKLOADS = {
    "cfg2_64x64_K32": lambda: otinputs.config_marginals(2),
    "bg_32x32_K16": lambda: (32, 16) + otinputs.mixture_pair(32, 5, 3, background=1e-3),
}
# direct solver of the Newton systems (oracle.ipm.newton_step): at 64^2,
# K = 32 the sparse LU of the full saddle system does not finish in hours,
# the potential-only elimination takes about 30 s per system
DIRECT = {"cfg2_64x64_K32": "reduced", "bg_32x32_K16": "saddle"}


def make(name):
    n, K, ri, rf = WORKLOADS[name]()
    prob = Problem(structured_mesh(n), K, ri, rf)
    t0 = time.perf_counter()
    r = solve_ipm(prob, tol=1e-6, final_tol=1e-10, max_newton=40, direct=DIRECT[name])
    dt = time.perf_counter() - t0
    if not r.converged:
        raise RuntimeError(f"oracle did not converge on {name}")
    path = os.path.join(HERE, f"oracle_{name}.npz")
    meta = dict(n=n, K=K, tol=1e-6, final_tol=1e-10, direct=DIRECT[name], mu=r.mu, cost=r.cost, dual=r.dual, gap=r.gap,
                newton_per_mu=[int(c) for c in r.newton_per_mu], seconds=dt)
    np.savez_compressed(path, rho=r.rho.ravel(), phi=r.phi.ravel(), meta=json.dumps(meta))
    print(name, json.dumps(meta), flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(WORKLOADS)):
        make(nm)
