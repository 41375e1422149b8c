"""Long-horizon parity at the full workload size, in the solver settings that
bench.py times: 500 Newmark steps of the 256x256, P = 35 problem (8x8
subdomains) against the oracle's stored mean and standard deviation at steps
2, 10, 50, 100, 200, 300, 400 and 500 (tests/golden/cfg2_oracle.txt, written
by tests/golden/make_golden.py from the oracle alone).

Bound: relative L2 error <= 1e-6 of both moment fields over the stored
sub-grid (every 16th node in each direction, 289 nodes), and of their
full-field L2 norms, at every recorded step.
"""

import numpy as np
import pytest

import golden_cfg2
import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_cfg2_500_steps_within_1e6(precision):
    import bench
    import paper_2512_23027_amd as sgw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    gold = golden_cfg2.load()
    sub = golden_cfg2.subgrid(256)
    s = sgw.Solver(workloads.config("cfg2"), **bench.solver_settings(precision))
    s.factor()
    s.autotune()
    s.set_state()
    done = 0
    worst = 0.0
    for step in sorted(gold):
        st = s.step(step - done)
        assert st["status"] == 0
        done = step
        m, v = s.moments()
        m = m.cpu().numpy()
        sd = np.sqrt(v.cpu().numpy())
        nm, ns, gm, gs = gold[step]
        errs = (np.linalg.norm(m[sub] - gm) / np.linalg.norm(gm),
                np.linalg.norm(sd[sub] - gs) / np.linalg.norm(gs),
                abs(np.linalg.norm(m) - nm) / nm, abs(np.linalg.norm(sd) - ns) / ns)
        print("step %d errors %s" % (step, " ".join("%.2e" % e for e in errs)), flush=True)
        worst = max(worst, max(errs))
    s.close()
    assert worst <= 1e-6, worst
