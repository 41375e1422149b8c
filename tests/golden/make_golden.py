"""Write oracle reference values for the long-horizon parity tests.

Calls only ``oracle/`` (and the seeded workload definitions).  For the
256x256, P = 35 workload it runs the oracle (CG with the mean-matrix
preconditioner to 1e-14 per step) and stores, at the recorded steps, the mean
and standard-deviation fields on the sub-grid of every 16th mesh node in each
direction, plus the full-field L2 norms.  Output: cfg2_oracle.txt (text).

Usage: python tests/golden/make_golden.py [nsteps]
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle.sg import SGProblem  # noqa: E402

STRIDE = 16


def subgrid(n):
    idx = np.arange(0, n + 1, STRIDE)
    return (idx[None, :] + (n + 1) * idx[:, None]).ravel()


def main():
    nsteps = int(sys.argv[1]) if len(sys.argv) > 1 else 500
    record = {2, 10, 50, 100, 200, 300, 400, 500}
    prm = workloads.config("cfg2")
    pr = SGProblem(prm, solver="cg")
    sub = subgrid(prm["n"])
    out_path = os.path.join(HERE, "cfg2_oracle.txt")
    U, V, A = pr.initial_state()
    lines = ["# oracle reference for cfg2 (256x256, P=35, dt 1e-3), written by make_golden.py",
             "# sub-grid: mesh nodes (16i, 16j); per recorded step: 'step s norm_mean norm_std'",
             "# then one line per sub-grid node: 'mean std'"]
    t0 = time.time()
    for s in range(1, nsteps + 1):
        U, V, A = pr.step(U, V, A)
        if s in record:
            mean, std = pr.moments(U)
            lines.append("step %d %.17e %.17e" % (s, np.linalg.norm(mean), np.linalg.norm(std)))
            lines.extend("%.17e %.17e" % (mean[v], std[v]) for v in sub)
            with open(out_path, "w") as f:
                f.write("\n".join(lines) + "\n")
            print("step %d written (%.0f s)" % (s, time.time() - t0), flush=True)


if __name__ == "__main__":
    main()
