"""Several independent problems in one call (sgw_step_batch): uneven seeded
rectilinear partitions (the structure of the batched workload, at sizes the
oracle finishes quickly), different variances and correlation lengths.  The
batched states equal the one-at-a-time states bit for bit (same kernels,
same order inside each problem), and each problem matches the oracle."""

import numpy as np
import pytest

import workloads
from oracle.sg import SGProblem, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problems():
    out = []
    for p in range(3):
        rng = np.random.default_rng(700 + p)
        xs, ys = workloads.random_splits(rng, 48, counts=(3, 4), min_cells=6)
        out.append(workloads.config("cfg1", n=48, xsplits=xs, ysplits=ys,
                                    sigma=float(rng.uniform(0.1, 0.4)),
                                    bx=float(rng.uniform(0.2, 0.6)), by=float(rng.uniform(0.2, 0.6)),
                                    x0=float(rng.uniform(0.3, 0.7)), y0=float(rng.uniform(0.3, 0.7))))
    return out


@pytest.mark.parametrize("inner", [0, 1])
def test_batch_equals_sequential_and_oracle(inner):
    import paper_2512_23027_amd as sgw
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prms = _problems()
    nsteps = 12

    def make():
        ss = []
        for prm in prms:
            s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14, inner_prec=inner)
            s.factor()
            s.set_state()
            ss.append(s)
        return ss

    seq = make()
    for s in seq:
        assert s.step(nsteps)["status"] == 0
    bat = make()
    stats = sgw.step_batch(bat, nsteps)
    assert all(st["status"] == 0 and st["steps"] == nsteps for st in stats)
    for a, b, prm in zip(seq, bat, prms):
        ua, ub = a.get_state()[0], b.get_state()[0]
        assert torch.equal(ua, ub)
        ref = SGProblem(prm)
        U, V, A = ref.initial_state()
        for _ in range(nsteps):
            U, V, A = ref.step(U, V, A)
        m, sd = ref.moments(U)
        mg, vg = b.moments()
        assert rel_l2(mg.cpu().numpy(), m) < 1e-10
        assert rel_l2(np.sqrt(vg.cpu().numpy()), sd) < 1e-10
    for s in seq + bat:
        s.close()


def test_batch_rejects_repeated_context():
    import paper_2512_23027_amd as sgw
    s = sgw.Solver(_problems()[0])
    s.factor()
    s.set_state()
    with pytest.raises(sgw.SGWError):
        sgw.step_batch([s, s], 1)
    s.close()
