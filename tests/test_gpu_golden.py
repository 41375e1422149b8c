"""Long-horizon and full-size parity against stored oracle runs
(tests/golden/<workload>_oracle.npz, written by tests/golden/make_golden.py
from the oracle alone), in the solver settings that bench.py times, compared
over every mesh node:
* 500 Newmark steps of the 256x256, P = 35 workload (8x8 subdomains) at
  steps 2, 10, 25, 100, 200 and 500, both timed stacks;
* the first 20 steps of the 512x512, P = 165 workload (16x16 subdomains,
  43.1 M SG unknowns) at steps 2, 10 and 20, the full stack.
Bound: relative L2 error <= 1e-6 of the mean and of the standard deviation
at every stored step.
"""

import numpy as np
import pytest

import golden_io
import workloads
from oracle.sg import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _check(name, precision):
    import bench
    import paper_2512_23027_amd as sgw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    gold, _ = golden_io.load(name)
    if not gold:
        pytest.skip("no stored oracle run for %s" % name)
    s = sgw.Solver(workloads.config(name), **bench.solver_settings(precision))
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
        gm, gs = gold[step]
        em = rel_l2(m.cpu().numpy(), gm)
        es = rel_l2(np.sqrt(v.cpu().numpy()), gs)
        print("%s %s step %d errors %.2e %.2e" % (name, precision, step, em, es), flush=True)
        worst = max(worst, em, es)
    s.close()
    assert worst <= 1e-6, worst


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_cfg2_500_steps_within_1e6(precision):
    _check("cfg2", precision)


def test_cfg5_20_steps_within_1e6():
    _check("cfg5", "mixed")
