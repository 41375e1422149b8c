"""The learned initial guess on the GPU: the network's MFMA forward and
backward kernels against the numpy reference (oracle/mlp.py, same bfloat16
operand rounding, float64 accumulation), Adam training, and the solver with
SGW_GUESS_LEARNED on the 32x32, P = 6 problem: trained on trajectories of the
training seeds, run on held-out seeds, its results match the oracle to the
same bound as the other guesses (1e-10 at rtol 1e-12, the FP64 bound) and
the iterations it saves are reported.

Tolerances: forward and gradient relative L2 error <= 2e-3 (a float32
intermediate that falls next to a bfloat16 rounding boundary may round the
other way than its float64 twin, a one-ulp (0.4 %) change of one operand).
"""

import numpy as np
import pytest

import workloads
from oracle import mlp as ref
from oracle.sg import SGProblem, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sgw():
    import paper_2512_23027_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("ng,H,nb", [(61, 256, 6), (61, 256, 300), (7, 40, 33)])
def test_forward_and_gradient_match_reference(sgw, ng, H, nb):
    m = sgw.GuessModel(ng, H, seed=11)
    w = m.params().cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(nb)
    x = rng.standard_normal((nb, 4 * ng)).astype(np.float32)
    t = (0.1 * rng.standard_normal((nb, ng))).astype(np.float32)
    y = m.forward(torch.from_numpy(x)).cpu().numpy()
    yr, _ = ref.forward(w, x, ng, H, bf16=True)
    assert _rel(y, yr) <= 2e-3
    loss, g = m.loss_grad(torch.from_numpy(x), torch.from_numpy(t))
    lr_, gr = ref.loss_grad(w, x, t, ng, H, bf16=True)
    assert abs(loss - lr_) <= 2e-3 * lr_
    g = g.cpu().numpy()
    W1, b1, W2, b2, W3, b3 = ref.unpack(np.arange(w.size), ng, H)
    for part in (W1, b1, W2, b2, W3, b3):  # every block of the gradient
        idx = part.ravel().astype(np.int64)
        assert _rel(g[idx], gr[idx]) <= 2e-3
    m.close()


def test_params_roundtrip_and_training_reduces_loss(sgw):
    ng, H = 16, 64
    m = sgw.GuessModel(ng, H, seed=3)
    w0 = m.params()
    m.set_params(w0 * 0.5)
    assert torch.equal(m.params(), w0 * 0.5)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((2048, 4 * ng)).astype(np.float32)
    A = rng.standard_normal((4 * ng, ng)) / np.sqrt(4 * ng)
    t = np.tanh(x @ A).astype(np.float32)   # a smooth teacher
    xt, tt = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    l0, _ = m.loss_grad(xt[:256], tt[:256])
    lf = m.train(xt, tt, epochs=40, batch=128, lr=2e-3, seed=1)
    l1, _ = m.loss_grad(xt[:256], tt[:256])
    assert np.isfinite(lf) and l1 < 0.2 * l0, (l0, l1, lf)
    m.close()


def _run(sgw, prm, nsteps, guess, model=None, record=None):
    s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14, guess=guess)
    s.factor()
    s.set_state()
    if model is not None:
        s.set_guess_model(model)
    if record is not None:
        s.record_guess_samples(*record)
    st = s.step(nsteps)
    m, v = s.moments()
    out = (st, m.cpu().numpy(), np.sqrt(v.cpu().numpy()), s.recorded_samples(),
           s.guess_fallbacks())
    s.record_guess_samples()
    s.close()
    return out


def test_learned_guess_trained_on_own_trajectories(sgw):
    train_seeds, test_seeds = workloads.learned_guess_seeds()
    nsteps = 200
    prm0 = workloads.cfg4(train_seeds[0])
    probe = sgw.Solver(prm0)
    ng, P = probe.ninterface, probe.P
    probe.close()
    cap = len(train_seeds) * nsteps * P
    X = torch.empty(cap, 4 * ng, dtype=torch.float32, device="cuda")
    T = torch.empty(cap, ng, dtype=torch.float32, device="cuda")
    n = 0
    for sd in train_seeds:
        st, _, _, cnt, _ = _run(sgw, workloads.cfg4(sd), nsteps, sgw.SGW_GUESS_NEWMARK,
                                record=(X[n:], T[n:]))
        assert cnt == (nsteps - 3) * P, cnt
        n += cnt
    model = sgw.GuessModel(ng, 256, seed=7)
    loss = model.train(X[:n], T[:n], epochs=60, batch=256, lr=1e-3, seed=2)
    assert np.isfinite(loss)
    its = {"prev": 0, "newmark": 0, "learned": 0}
    for sd in test_seeds:
        prm = workloads.cfg4(sd, nsteps=40)
        ref = SGProblem(prm)
        U, V, A = ref.initial_state()
        for _ in range(40):
            U, V, A = ref.step(U, V, A)
        mo, so = ref.moments(U)
        for name, g in (("prev", sgw.SGW_GUESS_PREV), ("newmark", sgw.SGW_GUESS_NEWMARK),
                        ("learned", sgw.SGW_GUESS_LEARNED)):
            st, m, sd_, _, fb = _run(sgw, prm, 40, g, model=model)
            assert st["status"] == 0
            assert rel_l2(m, mo) < 1e-10 and rel_l2(sd_, so) < 1e-10, (name, sd)
            its[name] += st["outer_iters"]
    print("outer PCG iterations over %d held-out runs x 40 steps: %s (training loss %.3e)"
          % (len(test_seeds), its, loss))
    model.close()
