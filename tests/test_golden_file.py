"""The stored oracle values of the 256x256, P = 35 workload are what the
oracle computes now: the first recorded step is recomputed (CPU, ~10 s)."""

import numpy as np

import golden_cfg2
import workloads
from oracle.sg import SGProblem


def test_golden_file_layout():
    g = golden_cfg2.load()
    assert sorted(g) == [2, 10, 50, 100, 200, 300, 400, 500]
    for nm, ns, m, s in g.values():
        assert m.shape == s.shape == (17 * 17,)
        assert nm > 0 and ns > 0 and np.all(s >= 0)


def test_golden_step2_matches_oracle():
    g = golden_cfg2.load()
    pr = SGProblem(workloads.config("cfg2"), solver="cg")
    U, V, A = pr.initial_state()
    for _ in range(2):
        U, V, A = pr.step(U, V, A)
    m, s = pr.moments(U)
    nm, ns, gm, gs = g[2]
    sub = golden_cfg2.subgrid(256)
    assert np.allclose(m[sub], gm, rtol=1e-10, atol=1e-14 * np.abs(gm).max())
    assert np.allclose(s[sub], gs, rtol=1e-10, atol=1e-14 * np.abs(gs).max())
    assert abs(np.linalg.norm(m) - nm) <= 1e-10 * nm
    assert abs(np.linalg.norm(s) - ns) <= 1e-10 * ns
