"""Pins for the oracle's FEM, Newmark stepping and SG system.

* P1 stiffness on the structured mesh reduces to the textbook 5-point
  Laplacian for a constant coefficient; the consistent mass integrates to the
  area; the full stiffness annihilates constants.
* Newmark average acceleration is the trapezoidal rule on (u, v): for one
  degree of freedom it must equal the Cayley transform
  (I - hA/2)^{-1} (I + hA/2) of A = [[0, 1], [-k/m, -c/m]], and for c = 0
  it gives u_n = cos(n theta) with tan(theta/2) = omega dt / 2.
* The 2-D deterministic problem of the paper's verification appendix
  (u0 = sin(2 pi x) sin(pi y), c = 1, f = 0, undamped) has the closed-form
  solution sin(2 pi x) sin(pi y) cos(pi sqrt(5) t); the oracle converges to it
  at second order in h and dt.
* sigma = 0: all PCE modes >= 1 stay exactly zero and mode 0 equals the
  deterministic run.
* Undamped, f = 0: the discrete energy 1/2 V'MV + 1/2 U'KU is conserved.
* The SG moments converge to the exact moments of the log-normal problem
  computed by tensor Gauss-Hermite quadrature over deterministic solves
  (the exact exp(sum g_l xi_l), no PCE), and agree with Monte Carlo within
  its standard error.
* Direct and mean-preconditioned CG solves agree.
* The premise of the forced-failure GPU test: on a 16x16 mesh (L = 2, input
  order 2) the SG transient matrix is positive definite at sigma = 0.2, and
  indefinite at sigma = 3, dt = 1, where the second-order truncation of
  exp(sigma xi), e^(sigma^2/2) (1 + sigma xi + sigma^2 (xi^2 - 1) / 2), is
  negative near xi = -1/sigma and the stiffness outweighs the mass term.
"""

import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla
from numpy.polynomial import hermite_e as He

from oracle.fem import StructuredMesh, assemble
from oracle.kle import kle_fields
from oracle.newmark import newmark_step
from oracle.sg import SGProblem, energy, rel_l2

BASE = dict(n=8, L=2, sigma=0.3, bx=0.5, by=0.5, p_in=2, p_out=2, dt=0.01,
            alpha0=0.0, alpha1=0.0, x0=0.5, y0=0.5, width=0.2, amp=1.0)


def test_fem_stencil_and_mass():
    mesh = StructuredMesh(6)
    K, M = assemble(mesh, np.ones((1, len(mesh.tris))))
    K = K[0].toarray()
    assert abs(M.sum() - 1.0) < 1e-14
    np.testing.assert_allclose(K @ np.ones(mesh.nn), 0.0, atol=1e-13)
    n = 6
    for j in range(1, n):
        for i in range(1, n):
            r = i + (n + 1) * j
            row = np.zeros(mesh.nn)
            row[r] = 4.0
            for d in (1, -1, n + 1, -(n + 1)):
                row[r + d] = -1.0
            np.testing.assert_allclose(K[r], row, atol=1e-14)


def _cayley(m, c, k, h, y):
    A = np.array([[0.0, 1.0], [-k / m, -c / m]])
    I2 = np.eye(2)
    return np.linalg.solve(I2 - 0.5 * h * A, (I2 + 0.5 * h * A) @ y)


@pytest.mark.parametrize("c", [0.0, 0.3])
def test_newmark_is_trapezoidal_rule(c):
    m, k, h = 2.0, 5.0, 0.07
    u, v = np.array([0.7]), np.array([-0.2])
    a = np.array([(-c * v[0] - k * u[0]) / m])
    y = np.array([u[0], v[0]])
    for _ in range(50):
        u, v, a = newmark_step(
            u, v, a, h, lambda x: m * x, lambda x: c * x,
            lambda f, _u: f / (m / (0.25 * h * h) + 0.5 * c / (0.25 * h) + k))
        y = _cayley(m, c, k, h, y)
        assert abs(u[0] - y[0]) < 1e-13 and abs(v[0] - y[1]) < 1e-13
    if c == 0.0:
        # undamped: rotation by theta in (u, v/omega), tan(theta/2) = omega h/2
        w = math.sqrt(k / m)
        theta = 2 * math.atan(w * h / 2)
        exact = 0.7 * math.cos(50 * theta) + (-0.2 / w) * math.sin(50 * theta)
        assert abs(u[0] - exact) < 1e-12


def _analytic_run(n, dt, T):
    mesh = StructuredMesh(n)
    u0 = np.sin(2 * np.pi * mesh.x) * np.sin(np.pi * mesh.y)
    prm = dict(n=n, L=0, sigma=0.0, bx=1.0, by=1.0, p_in=0, p_out=0, dt=dt,
               alpha0=0.0, alpha1=0.0, u0=u0)
    pr = SGProblem(prm)
    nsteps = int(round(T / dt))
    out = pr.run(nsteps, record={nsteps})
    exact = u0 * math.cos(math.pi * math.sqrt(5.0) * nsteps * dt)
    return rel_l2(out[nsteps][0], exact)


def test_analytic_solution_second_order():
    T = 0.4
    e1 = _analytic_run(16, T / 40, T)
    e2 = _analytic_run(32, T / 80, T)
    e3 = _analytic_run(64, T / 160, T)
    assert e1 < 0.05
    assert 3.3 < e1 / e2 < 4.7 and 3.3 < e2 / e3 < 4.7, (e1, e2, e3)


def test_sigma_zero_reduces_to_deterministic():
    prm = dict(BASE, sigma=0.0, p_out=3, alpha0=0.5445, alpha1=0.0174)
    sg = SGProblem(prm)
    U, V, A = sg.initial_state()
    det = SGProblem(dict(prm, L=0, p_in=0, p_out=0))
    u, v, a = det.initial_state()
    for _ in range(15):
        U, V, A = sg.step(U, V, A)
        u, v, a = det.step(u, v, a)
    assert np.all(U[:, 1:] == 0.0)
    np.testing.assert_allclose(U[:, 0], u[:, 0], rtol=0, atol=1e-14)


def test_energy_conservation_undamped():
    sg = SGProblem(dict(BASE, p_out=3))
    U, V, A = sg.initial_state()
    e0 = energy(sg, U, V)
    for _ in range(60):
        U, V, A = sg.step(U, V, A)
        assert abs(energy(sg, U, V) - e0) <= 1e-12 * e0


def test_direct_and_cg_agree():
    prm = dict(BASE, n=16, p_out=3, alpha0=0.5445, alpha1=0.0174, dt=0.005)
    a = SGProblem(prm, solver="direct").run(20, record={20})
    b = SGProblem(prm, solver="cg").run(20, record={20})
    assert rel_l2(b[20][0], a[20][0]) < 1e-12
    assert rel_l2(b[20][1], a[20][1]) < 1e-10


def _det_solve_samples(prm, xis, nsteps):
    """Deterministic runs with the exact log-normal coefficient exp(g . xi)."""
    mesh = StructuredMesh(prm["n"])
    g = kle_fields(prm["sigma"], prm["bx"], prm["by"], prm["L"], mesh.cx, mesh.cy)
    f = mesh.free
    r2 = (mesh.x - prm["x0"]) ** 2 + (mesh.y - prm["y0"]) ** 2
    u0 = prm["amp"] * np.exp(-r2 / prm["width"] ** 2)
    _, Mall = assemble(mesh, np.ones((1, len(mesh.tris))))
    M = Mall[f][:, f].tocsc()
    dt, z, gm = prm["dt"], 0.25, 0.5
    a0, a1 = prm["alpha0"], prm["alpha1"]
    out = []
    for xi in xis:
        coef = np.exp(xi @ g)[None, :]
        Kall, _ = assemble(mesh, coef)
        K = Kall[0][f][:, f].tocsc()
        C = (a0 * M + a1 * K).tocsc()
        lu = spla.splu((M / (z * dt * dt) + gm * C / (z * dt) + K).tocsc())
        u = u0[f].copy()
        v = np.zeros_like(u)
        a = spla.splu(M).solve(-(K @ u))
        for _ in range(nsteps):
            u, v, a = newmark_step(u, v, a, dt, lambda x: M @ x,
                                   lambda x: C @ x, lambda F, _u: lu.solve(F))
        out.append(u)
    return np.array(out)


def test_sg_converges_to_gauss_hermite_moments():
    prm = dict(BASE, alpha0=0.5445, alpha1=0.0174)
    nsteps = 25
    x, w = He.hermegauss(14)
    w = w / math.sqrt(2 * math.pi)
    xis = np.array([(a, b) for a in x for b in x])
    wts = np.array([wa * wb for wa in w for wb in w])
    u = _det_solve_samples(prm, xis, nsteps)
    mean_ex = wts @ u
    std_ex = np.sqrt(np.maximum(wts @ (u * u) - mean_ex ** 2, 0.0))
    errs = []
    for p in (1, 2, 3, 4):
        sg = SGProblem(dict(prm, p_in=2 * p, p_out=p))
        U, V, A = sg.initial_state()
        for _ in range(nsteps):
            U, V, A = sg.step(U, V, A)
        m = U[:, 0]
        s = np.sqrt(np.sum(U[:, 1:] ** 2, axis=1))
        errs.append((rel_l2(m, mean_ex), rel_l2(s, std_ex)))
    em = [e[0] for e in errs]
    es = [e[1] for e in errs]
    assert em[-1] < 1e-6 and es[-1] < 1e-4, errs
    for i in range(3):
        assert em[i + 1] < 0.5 * em[i] and es[i + 1] < 0.5 * es[i], errs


def test_sg_mean_within_monte_carlo_error():
    prm = dict(BASE, alpha0=0.5445, alpha1=0.0174)
    nsteps = 25
    rng = np.random.default_rng(11)
    ns = 1000
    u = _det_solve_samples(prm, rng.standard_normal((ns, 2)), nsteps)
    mc_mean = u.mean(axis=0)
    se = u.std(axis=0, ddof=1) / math.sqrt(ns)
    sg = SGProblem(dict(prm, p_in=4, p_out=3))
    U, V, A = sg.initial_state()
    for _ in range(nsteps):
        U, V, A = sg.step(U, V, A)
    z = np.abs(U[:, 0] - mc_mean) / np.maximum(se, 1e-300)
    assert np.max(z) < 4.5


# ---------------------------------------------------------------------------
# Random initial conditions (Eq. acous_sto: u_0(x, theta), v_0(x, theta)),
# given by their chaos coefficients u0_modes / v0_modes.
# ---------------------------------------------------------------------------
def _pulse(prm, mesh):
    r2 = (mesh.x - prm["x0"]) ** 2 + (mesh.y - prm["y0"]) ** 2
    return prm["amp"] * np.exp(-r2 / prm["width"] ** 2)


def test_random_initial_condition_sigma_zero_is_linear():
    # c_s deterministic: every chaos mode evolves on its own, so the modes of
    # u_0 = (1 + d xi_1) pulse and v_0 = e xi_2 pulse are d and e times
    # deterministic runs (a transposed or misplaced mode fails)
    d, e = 0.3, 0.7
    prm = dict(BASE, sigma=0.0, p_out=2, alpha0=0.5445, alpha1=0.0174)
    mesh = StructuredMesh(prm["n"])
    pulse = _pulse(prm, mesh)
    P = 6
    u0 = np.zeros((P, mesh.nn))
    v0 = np.zeros((P, mesh.nn))
    u0[0], u0[1], v0[2] = pulse, d * pulse, e * pulse  # modes 1, 2 = xi_1, xi_2
    sg = SGProblem(dict(prm, u0_modes=u0, v0_modes=v0))
    U, V, A = sg.initial_state()
    det = SGProblem(dict(prm, L=0, p_in=0, p_out=0))
    u, v, a = det.initial_state()
    dv = SGProblem(dict(prm, L=0, p_in=0, p_out=0, u0=0 * pulse, v0_modes=pulse[None, :]))
    uv, vv, av = dv.initial_state()
    for _ in range(12):
        U, V, A = sg.step(U, V, A)
        u, v, a = det.step(u, v, a)
        uv, vv, av = dv.step(uv, vv, av)
    np.testing.assert_allclose(U[:, 0], u[:, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(U[:, 1], d * u[:, 0], rtol=0, atol=1e-14)
    np.testing.assert_allclose(U[:, 2], e * uv[:, 0], rtol=0, atol=1e-14)
    assert np.all(U[:, 3:] == 0.0)


def test_random_initial_condition_vs_gauss_hermite():
    # random medium and random initial pressure and velocity: the SG
    # moments converge to the tensor Gauss-Hermite moments of deterministic
    # runs with the exact coefficient exp(g . xi) and the sampled initial
    # state u_0 = (1 + d xi_1) pulse, v_0 = e xi_2 pulse
    d, e = 0.4, 2.0
    prm = dict(BASE, alpha0=0.5445, alpha1=0.0174)
    nsteps = 25
    mesh = StructuredMesh(prm["n"])
    pulse = _pulse(prm, mesh)
    g = kle_fields(prm["sigma"], prm["bx"], prm["by"], prm["L"], mesh.cx, mesh.cy)
    f = mesh.free
    _, Mall = assemble(mesh, np.ones((1, len(mesh.tris))))
    M = Mall[f][:, f].tocsc()
    dt, z, gm = prm["dt"], 0.25, 0.5
    x, w = He.hermegauss(14)
    w = w / math.sqrt(2 * math.pi)
    us, wts = [], []
    for ia, xa in enumerate(x):
        for ib, xb in enumerate(x):
            xi = np.array([xa, xb])
            Kall, _ = assemble(mesh, np.exp(xi @ g)[None, :])
            K = Kall[0][f][:, f].tocsc()
            C = (prm["alpha0"] * M + prm["alpha1"] * K).tocsc()
            lu = spla.splu((M / (z * dt * dt) + gm * C / (z * dt) + K).tocsc())
            u = (1 + d * xa) * pulse[f]
            v = e * xb * pulse[f]
            a = spla.splu(M).solve(-(K @ u) - C @ v)
            for _ in range(nsteps):
                u, v, a = newmark_step(u, v, a, dt, lambda q: M @ q, lambda q: C @ q,
                                       lambda F, _u: lu.solve(F))
            us.append(u)
            wts.append(w[ia] * w[ib])
    us, wts = np.array(us), np.array(wts)
    mean_ex = wts @ us
    std_ex = np.sqrt(np.maximum(wts @ (us * us) - mean_ex ** 2, 0.0))
    errs = []
    for p in (2, 4):
        from oracle.pce import pce_size
        P = pce_size(2, p)
        u0 = np.zeros((P, mesh.nn))
        v0 = np.zeros((P, mesh.nn))
        u0[0], u0[1], v0[2] = pulse, d * pulse, e * pulse
        sg = SGProblem(dict(prm, p_in=2 * p, p_out=p, u0_modes=u0, v0_modes=v0))
        U, V, A = sg.initial_state()
        for _ in range(nsteps):
            U, V, A = sg.step(U, V, A)
        errs.append((rel_l2(U[:, 0], mean_ex), rel_l2(np.sqrt(np.sum(U[:, 1:] ** 2, axis=1)),
                                                       std_ex)))
    # measured: p = 2: 9.4e-5 / 2.2e-3, p = 4: 4.3e-7 / 2.5e-5 (mean / std)
    assert errs[1][0] < 2e-6 and errs[1][1] < 1e-4, errs
    assert errs[1][0] < 0.1 * errs[0][0] and errs[1][1] < 0.1 * errs[0][1], errs


def test_truncated_pce_indefinite_premise():
    import workloads
    # the 1-D truncation takes the value (1 - sigma^2) / 2 e^(sigma^2/2) at its minimum
    sig = 3.0
    xi = -1.0 / sig
    f = math.exp(sig * sig / 2) * (1 + sig * xi + sig * sig * (xi * xi - 1) / 2)
    assert f < 0 and abs(f - (1 - sig * sig) / 2 * math.exp(sig * sig / 2)) < 1e-9 * abs(f)
    lo = {}
    for sigma, dt in ((0.2, 0.005), (3.0, 1.0)):
        prm = workloads.config("cfg1", n=16, xsplits=workloads.uniform_splits(16, 2),
                               ysplits=workloads.uniform_splits(16, 2), sigma=sigma, dt=dt)
        K = SGProblem(prm).assembled_Kt()
        lo[sigma] = float(spla.eigsh(K, k=1, which="SA", return_eigenvectors=False)[0])
    assert lo[0.2] > 0 and lo[3.0] < -10, lo
