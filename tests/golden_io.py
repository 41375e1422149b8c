"""Reader of tests/golden/cfg2_oracle.txt (oracle mean and standard deviation
of the 256x256, P = 35 workload at recorded steps, on the sub-grid of every
16th mesh node; written by tests/golden/make_golden.py)."""

import os

import numpy as np

PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cfg2_oracle.txt")
STRIDE = 16


def subgrid(n):
    idx = np.arange(0, n + 1, STRIDE)
    return (idx[None, :] + (n + 1) * idx[:, None]).ravel()


def load():
    """{step: (norm_mean, norm_std, mean[sub], std[sub])}"""
    out = {}
    cur = None
    for line in open(PATH):
        if line.startswith("#"):
            continue
        f = line.split()
        if f[0] == "step":
            cur = int(f[1])
            out[cur] = (float(f[2]), float(f[3]), [], [])
        else:
            out[cur][2].append(float(f[0]))
            out[cur][3].append(float(f[1]))
    return {s: (a, b, np.array(m), np.array(d)) for s, (a, b, m, d) in out.items()}
