"""Reader of the stored oracle runs (tests/golden/<workload>_oracle.npz,
written by tests/golden/make_golden.py from the oracle alone): the mean and
standard-deviation fields over all mesh nodes at the stored steps."""

import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name="cfg2"):
    """{step: (mean, std)} (float64 arrays over all (n+1)^2 nodes) and the
    mesh size n; an empty dict if the file is missing."""
    path = os.path.join(HERE, "%s_oracle.npz" % name)
    if not os.path.exists(path):
        return {}, None
    z = np.load(path, allow_pickle=False)
    out = {int(s): (z["mean_%d" % s].astype(np.float64), z["std_%d" % s].astype(np.float64))
           for s in z["steps"]}
    return out, int(z["n"])
