"""The batched workload at its real size: two of its eight problems (384x384
meshes, P = 84, seeded uneven rectilinear splits, 0.5-2x cell areas)
advanced together by sgw_step_batch in the timed solver settings (FP32
DD-PCG inside FP64 refinement, Chebyshev subdomain preconditioner at
P = 84, the two output groups of the FP64 SG apply in the refinement
residual), compared over all mesh nodes with the stored oracle values at
steps 5 and 10 (tests/golden/cfg3-<p>_oracle.npz, written from the oracle
alone): relative L2 error of mean and standard deviation within 1e-6."""

import numpy as np
import pytest

import workloads
from golden_io import load
from oracle.sg import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_cfg3_batched_pair_within_1e6():
    import paper_2512_23027_amd as sgw
    import bench
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    names = ["cfg3-0", "cfg3-1"]
    gold = [load(nm)[0] for nm in names]
    ss = []
    for nm in names:
        s = sgw.Solver(workloads.config(nm), **bench.solver_settings("mixed"))
        print("%s: P=%d, %d subdomains" % (nm, s.P, s.nsub), flush=True)
        s.factor()
        s.set_state()
        ss.append(s)
    done = 0
    for step in (5, 10):
        st = sgw.step_batch(ss, step - done)
        done = step
        for nm, s, g, x in zip(names, ss, gold, st):
            assert x["status"] == 0
            m, v = s.moments()
            gm, gs = g[step]
            em, es = rel_l2(m.cpu().numpy(), gm), rel_l2(np.sqrt(v.cpu().numpy()), gs)
            print("%s step %d: errors %.2e %.2e" % (nm, step, em, es), flush=True)
            assert em < 1e-6 and es < 1e-6, (nm, step, em, es)
    for s in ss:
        s.close()
