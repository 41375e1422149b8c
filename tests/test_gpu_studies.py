"""One-GPU replicas of the paper's deterministic-medium studies, through the
C-ABI, with the oracle and the closed-form solution as references.

* Deterministic medium (L = 0, one chaos mode): trajectories of the FP64
  path match the oracle within 1e-10, the refinement path within 1e-6.
* Verification against the closed form of the deterministic appendix
  (u_0 = sin(2 pi x) sin(pi y), c = 1, f = 0, undamped:
  u = sin(2 pi x) sin(pi y) cos(pi sqrt(5) t)): second-order convergence in
  h and dt together, and the Courant-number study (Eq. CFL) on meshes of the
  paper's two sizes: at a fixed Courant number the error falls with the mesh,
  the largest Courant number (2) gives several times the error of 0.65 and
  its error grows with time, and 0.65 (the paper's choice) gives the
  smallest error of the four.
* Comparison with the one-level preconditioners (Sec. 6.1): on a
  deterministic 40 x 40 mesh (1,681 nodes; the paper's study has 1,563
  vertices) at dt = 0.01 (the paper's), 0.1 and 0.25, the average
  interface-PCG iterations per step with 4 to 64 subdomains: two-level NN <=
  one-level NN <= lumped throughout; at the large time step the one-level
  counts grow with the number of subdomains and the two-level ones stay
  nearly flat; every variant reaches the oracle's solution.
The tables are printed (pytest -s).
"""

import math

import numpy as np
import pytest

import workloads
from oracle.sg import SGProblem, rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sgw():
    import paper_2512_23027_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def _det(n, ns, dt, **over):
    p = dict(n=n, L=0, sigma=0.0, bx=1.0, by=1.0, p_in=0, p_out=0, dt=dt, alpha0=0.0,
             alpha1=0.0, x0=0.5, y0=0.5, width=0.1, amp=1.0,
             xsplits=workloads.uniform_splits(n, ns), ysplits=workloads.uniform_splits(n, ns))
    p.update(over)
    return p


def test_deterministic_trajectories_match_oracle(sgw):
    prm = _det(48, 3, 0.005, alpha0=workloads.ALPHA0, alpha1=workloads.ALPHA1, x0=0.4, y0=0.6)
    ref = SGProblem(prm)
    U, V, A = ref.initial_state()
    for _ in range(30):
        U, V, A = ref.step(U, V, A)
    mo, _ = ref.moments(U)
    for kw, tol in ((dict(), 1e-10),
                    (dict(precision=sgw.SGW_FP32_IR64, guess=sgw.SGW_GUESS_NEWMARK), 1e-6)):
        s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14, **kw)
        assert s.P == 1
        s.factor()
        s.set_state()
        st = s.step(30)
        m, v = s.moments()
        err = rel_l2(m.cpu().numpy(), mo)
        print("deterministic 48x48, %s: error %.2e, %.1f outer iterations per step"
              % ("FP64" if not kw else "refined FP32", err, st["outer_iters"] / 30))
        assert st["status"] == 0 and err < tol, err
        assert float(v.abs().max()) == 0.0
        s.close()


def _analytic_error(sgw, n, ns, dt, T, sample=None, relative=True):
    """Error against the closed form at T (and at the steps in sample):
    relative L2 (Eq. Norm), or with relative=False the L2 error over the
    norm of the initial state (free of the zero crossings of cos)."""
    prm = _det(n, ns, dt)
    s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14)
    s.factor()
    x = np.tile(np.arange(n + 1) / n, n + 1)
    y = np.repeat(np.arange(n + 1) / n, n + 1)
    shape = np.sin(2 * math.pi * x) * np.sin(math.pi * y)
    s.set_state(U=torch.from_numpy(shape[None, :].copy()))
    nsteps = int(round(T / dt))
    errs = {}
    done = 0
    for k in sorted(set((sample or []) + [nsteps])):
        s.step(k - done)
        done = k
        m, _ = s.moments()
        exact = shape * math.cos(math.pi * math.sqrt(5.0) * k * dt)
        m = m.cpu().numpy()
        errs[k] = (rel_l2(m, exact) if relative
                   else float(np.linalg.norm(m - exact) / np.linalg.norm(shape)))
    s.close()
    return errs[nsteps], errs


def test_closed_form_second_order(sgw):
    T = 0.4
    e = [_analytic_error(sgw, n, 4, T / (n * 5 / 2), T)[0] for n in (16, 32, 64)]
    print("closed form at t = 0.4, meshes 16, 32, 64 (dt = h / 2.5): errors %s" % e)
    assert e[0] < 0.05
    assert 3.3 < e[0] / e[1] < 4.7 and 3.3 < e[1] / e[2] < 4.7, e


def test_courant_number_study(sgw):
    # meshes of 117^2 = 13,689 nodes and 233^2 = 54,289 nodes (the paper's
    # 13,472 and 53,263 vertices), Courant numbers c dt / h up to 2, errors
    # over the initial amplitude at t = 0.125, 0.25, 0.5 s.  Measured with the
    # oracle on the coarse mesh: 3.3e-4 / 1.7e-4 / 2.1e-4 / 1.7e-3 at
    # t = 0.25 for C = 0.25 / 0.65 / 1 / 2: the consistent-mass P1 phase lead
    # and the Newmark period elongation partly cancel, so C = 0.65 (the
    # paper's choice) gives the smallest error, not the smallest C.
    T = 0.5
    courant = (0.25, 0.65, 1.0, 2.0)
    table = {}
    for n, ns in ((116, 4), (232, 8)):
        for cfl in courant:
            nsteps = int(round(T / (cfl / n)))
            e, series = _analytic_error(sgw, n, ns, T / nsteps, T,
                                        sample=[nsteps // 4, nsteps // 2], relative=False)
            table[(n, cfl)] = [series[k] for k in sorted(series)]
            print("Courant study: mesh %d^2, C = %.2f: error / |u_0| %s at t = 0.125, 0.25, 0.5"
                  % (n, cfl, " ".join("%.2e" % v for v in table[(n, cfl)])))
    for n in (116, 232):
        e = {c: table[(n, c)][1] for c in courant}
        assert e[2.0] > 3 * e[0.65] and e[0.65] <= min(e[0.25], e[1.0]), (n, e)
        early, mid, _ = table[(n, 2.0)]
        assert mid > 2 * early, (n, table[(n, 2.0)])  # the error grows with time
    for c in courant:
        assert table[(232, c)][1] < 0.4 * table[(116, c)][1], c


def _iterations(sgw, prm, precond, nsteps):
    s = sgw.Solver(prm, rtol=1e-8, inner_rtol=1e-12, precond=precond)
    s.factor()
    s.set_state()
    st = s.step(nsteps)
    assert st["status"] == 0
    m, _ = s.moments()
    s.close()
    return st["outer_iters"] / nsteps, m.cpu().numpy()


def test_one_level_preconditioners(sgw):
    """At the paper's dt = 0.01 on this mesh the stiffness term is about 4 %
    of the mass term M / (zeta dt^2), which dominates even at the scale of
    the largest subdomains, so every variant converges in 3-5 iterations and
    the coarse space matters little; the growth with the number of
    subdomains that the paper reports appears as the stiffness gains on the
    mass term at the subdomain scale (H^2 approaching zeta c dt^2), here at
    dt = 0.1 and 0.25, where the one-level counts grow several times faster
    than the two-level ones."""
    nsteps = 20
    names = {sgw.SGW_PRECOND_NN2: "two-level NN", sgw.SGW_PRECOND_NN1: "one-level NN",
             sgw.SGW_PRECOND_LUMPED: "lumped"}
    counts = (2, 4, 5, 8)
    table = {}
    for dt in (0.01, 0.1, 0.25):
        its = {k: [] for k in names}
        for ns in counts:
            prm = _det(40, ns, dt, x0=0.37, y0=0.58, width=0.15)
            ref = SGProblem(prm)
            U, V, A = ref.initial_state()
            for _ in range(nsteps):
                U, V, A = ref.step(U, V, A)
            mo, _ = ref.moments(U)
            for pc in names:
                it, m = _iterations(sgw, prm, pc, nsteps)
                its[pc].append(it)
                assert rel_l2(m, mo) < 1e-6, (dt, ns, names[pc])
        table[dt] = its
        print("average interface PCG iterations per step, 40x40 mesh, dt %g, rtol 1e-8" % dt)
        print("subdomains:    " + " ".join("%6d" % (c * c) for c in counts))
        for pc, name in names.items():
            print("%-13s " % name + " ".join("%6.2f" % v for v in its[pc]))
        nn2, nn1, lump = its[sgw.SGW_PRECOND_NN2], its[sgw.SGW_PRECOND_NN1], \
            its[sgw.SGW_PRECOND_LUMPED]
        assert all(a <= b <= c for a, b, c in zip(nn2, nn1, lump)), its
    # measured at dt 0.25, 4 -> 64 subdomains: two-level 4.2 -> 9.0,
    # one-level 5.0 -> 20.0, lumped 17.6 -> 28.1 iterations per step
    big = table[0.25]
    nn2, nn1, lump = big[sgw.SGW_PRECOND_NN2], big[sgw.SGW_PRECOND_NN1], \
        big[sgw.SGW_PRECOND_LUMPED]
    assert nn1[-1] - nn1[0] > 2 * (nn2[-1] - nn2[0]), big
    assert lump[-1] > 1.3 * lump[0] and nn1[-1] > 2 * nn1[0], big


def test_random_initial_conditions(sgw):
    """Random initial pressure and velocity (Eq. acous_sto: u_0(x, theta),
    v_0(x, theta)) in a random medium, given by their chaos coefficients:
    u_0 = (1 + 0.4 xi_1) pulse, v_0 = 2 xi_2 pulse on the 32x32, P = 6
    problem.  The state is set through the C-ABI; the FP64 path matches the
    oracle within 1e-10, the refinement path within 1e-6."""
    prm = workloads.config("cfg1")
    n = prm["n"]
    x = np.tile(np.arange(n + 1) / n, n + 1)
    y = np.repeat(np.arange(n + 1) / n, n + 1)
    pulse = np.exp(-((x - 0.45) ** 2 + (y - 0.55) ** 2) / 0.1 ** 2)
    u0 = np.zeros((6, (n + 1) ** 2))
    v0 = np.zeros_like(u0)
    u0[0], u0[1], v0[2] = pulse, 0.4 * pulse, 2.0 * pulse
    ref = SGProblem(dict(prm, u0_modes=u0, v0_modes=v0))
    U, V, A = ref.initial_state()
    for _ in range(50):
        U, V, A = ref.step(U, V, A)
    mo, so = ref.moments(U)
    for kw, tol in ((dict(), 1e-10),
                    (dict(precision=sgw.SGW_FP32_IR64, guess=sgw.SGW_GUESS_NEWMARK), 1e-6)):
        s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14, **kw)
        s.factor()
        s.set_state(U=torch.from_numpy(u0), V=torch.from_numpy(v0))
        st = s.step(50)
        m, v = s.moments()
        em, es = rel_l2(m.cpu().numpy(), mo), rel_l2(np.sqrt(v.cpu().numpy()), so)
        print("random initial conditions, %s: errors %.2e %.2e"
              % ("FP64" if not kw else "refined FP32", em, es))
        assert st["status"] == 0 and em < tol and es < tol, (em, es)
        s.close()
