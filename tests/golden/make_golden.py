"""Write oracle reference values for the long-horizon parity tests.

Calls only ``oracle/`` (and the seeded workload definitions): the oracle
(CG with the mean-matrix preconditioner to a relative residual of 1e-14 per
step, no domain decomposition) advances the named workload and, at the
recorded steps, the full mean and standard-deviation fields over all
(n+1)^2 mesh nodes are stored in FP64 (numpy .npz, compressed).

* cfg2 (256x256, P = 35, 8x8 subdomains): steps 2, 10, 25, 100, 200, 500
  -> cfg2_oracle.npz (FP64)
* cfg5 (512x512, P = 165, 16x16 subdomains): the first 30 steps, stored at
  steps 2, 10, 20, 30 -> cfg5_oracle.npz (rounded to FP32: its parity bound
  is 1e-6 and FP32 keeps the stored fields within 6e-8 of the oracle's)
* cfg3-0, cfg3-1 (384x384, P = 84, seeded uneven splits; two of the eight
  problems of the batched workload): the first 10 steps, stored at steps 5
  and 10 -> cfg3-<p>_oracle.npz (FP32 as above)
The oracle's CG iteration count of every step is stored too (cg_iterations).

Usage: python tests/golden/make_golden.py cfg2|cfg5|cfg3-0|cfg3-1 [--out PATH]
       python tests/golden/make_golden.py cfg2|cfg5 --repack   (keep only the
       stored steps and precision above from a file written with more)
The file is rewritten after every recorded step (so a long run can be
inspected); --out writes elsewhere, to be moved into place when complete.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads  # noqa: E402
from oracle.sg import SGProblem  # noqa: E402

RECORD = {"cfg2": (2, 10, 25, 100, 200, 500),
          "cfg5": (2, 10, 20, 30), "cfg3-0": (5, 10), "cfg3-1": (5, 10)}
DTYPE = {"cfg2": np.float64, "cfg5": np.float32, "cfg3-0": np.float32, "cfg3-1": np.float32}


def save(path, name, n, fields, cg):
    steps = sorted(int(k[5:]) for k in fields if k.startswith("mean_"))
    keep = {k: np.asarray(v, dtype=DTYPE[name]) for k, v in fields.items()
            if int(k.split("_")[1]) in RECORD[name]}
    np.savez_compressed(path, steps=np.array([s for s in steps if s in RECORD[name]]),
                        n=np.array(n), cg_iterations=np.asarray(cg), **keep)


def repack(name):
    path = os.path.join(HERE, "%s_oracle.npz" % name)
    z = np.load(path, allow_pickle=False)
    fields = {k: z[k] for k in z.files if k.startswith(("mean_", "std_"))}
    cg = z["cg_iterations"] if "cg_iterations" in z.files else np.zeros(0)
    save(path, name, int(z["n"]), fields, cg)


def main():
    name = sys.argv[1]
    if "--repack" in sys.argv:
        repack(name)
        return
    record = RECORD[name]
    prm = workloads.config(name)
    pr = SGProblem(prm, solver="cg")
    out_path = os.path.join(HERE, "%s_oracle.npz" % name)
    if "--out" in sys.argv:
        out_path = sys.argv[sys.argv.index("--out") + 1]
    U, V, A = pr.initial_state()
    fields = {}
    t0 = time.time()
    for s in range(1, max(record) + 1):
        U, V, A = pr.step(U, V, A)
        print("step %d done (%.0f s, %d CG iterations)" % (s, time.time() - t0, pr.cg_iters[-1]),
              flush=True)
        if s in record:
            mean, std = pr.moments(U)
            fields["mean_%d" % s] = mean
            fields["std_%d" % s] = std
            save(out_path, name, prm["n"], fields, pr.cg_iters)


if __name__ == "__main__":
    main()
