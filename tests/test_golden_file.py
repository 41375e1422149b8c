"""The stored oracle runs are what the oracle computes now: their layout is
checked (the 256x256 run to step 500, the 512x512 run to step 30, two
384x384 problems of the batched set to step 10), and the first stored step
of the 256x256, P = 35 workload is recomputed here (CPU, ~15 s) and
compared over every node."""

import numpy as np

import golden_io
import workloads
from oracle.sg import SGProblem


def test_golden_file_layout():
    for name, n, steps, dtype_ok in (("cfg2", 256, [2, 10, 25, 100, 200, 500], True),
                                     ("cfg5", 512, [2, 10, 20, 30], True),
                                     ("cfg3-0", 384, [5, 10], True),
                                     ("cfg3-1", 384, [5, 10], True)):
        g, nn = golden_io.load(name)
        assert nn == n and sorted(g) == steps, (name, sorted(g))
        for m, s in g.values():
            assert m.shape == s.shape == ((n + 1) ** 2,)
            assert np.all(s >= 0) and np.linalg.norm(m) > 0 and np.linalg.norm(s) > 0


def test_golden_step2_matches_oracle():
    g, _ = golden_io.load("cfg2")
    pr = SGProblem(workloads.config("cfg2"), solver="cg")
    U, V, A = pr.initial_state()
    for _ in range(2):
        U, V, A = pr.step(U, V, A)
    m, s = pr.moments(U)
    gm, gs = g[2]
    assert np.linalg.norm(m - gm) <= 1e-10 * np.linalg.norm(gm)
    assert np.linalg.norm(s - gs) <= 1e-10 * np.linalg.norm(gs)
