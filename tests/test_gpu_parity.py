"""GPU parity of the HIP path (through the C-ABI) against the CPU oracle.

Tolerances (relative L2 over all mesh nodes, the error measure of Eq. Norm):
* SG operator apply, FP64: 1e-13 (one sparse contraction, rounding only);
* one SG solve at rtol 1e-12: 1e-10;
* trajectories on the FP64 path with rtol 1e-12: 1e-10 on the mean and the
  standard deviation at every 10th step (the bound for the FP64 path);
* zero variance: modes >= 1 stay exactly zero.
Sizes: the 32x32 problem (2x2 subdomains, ragged 64-row tails), an uneven
37x37 problem with 2x3 subdomains of different sizes, a 64x64 problem with
P = 35 (many waves, several K1 output groups), and the SG apply at the
full 256x256, P = 35 size.
"""

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


def _trajectory(sgw, prm, nsteps, rtol, every=10, prep=None, **kw):
    s = sgw.Solver(prm, rtol=rtol, inner_rtol=rtol * 1e-2, **kw)
    s.factor()
    if prep:
        prep(s)
    s.set_state()
    ref = SGProblem(prm)
    U, V, A = ref.initial_state()
    worst = (0.0, 0.0)
    stats = []
    for step in range(every, nsteps + 1, every):
        stats.append(s.step(every))
        for _ in range(every):
            U, V, A = ref.step(U, V, A)
        m, sd = ref.moments(U)
        mg, vg = s.moments()
        em = rel_l2(mg.cpu().numpy(), m)
        es = rel_l2(np.sqrt(vg.cpu().numpy()), sd)
        worst = (max(worst[0], em), max(worst[1], es))
    s.close()
    return worst, stats


def test_sg_apply_matches_oracle_cfg1(sgw):
    prm = workloads.config("cfg1")
    s = sgw.Solver(prm)
    ref = SGProblem(prm)
    g = torch.Generator().manual_seed(1)
    X = torch.randn(s.P, s.nn, dtype=torch.float64, generator=g)
    Y = s.apply_operator(X.cuda()).cpu().numpy()
    Yo = ref.apply_Kt(X.numpy()[:, ref.mesh.free].T)
    assert rel_l2(Y[:, ref.mesh.free].T, Yo) < 1e-13
    bnd = np.ones(s.nn, bool)
    bnd[ref.mesh.free] = False
    assert np.all(Y[:, bnd] == 0.0)
    s.close()


@pytest.mark.parametrize("n,ns,generic", [(64, 4, "0"), (64, 4, "1"), (256, 8, "0"),
                                          (256, 8, "1")])
def test_sg_apply_matches_oracle_p35(sgw, n, ns, generic, monkeypatch):
    """Both SG-apply kernels: the one with the unrolled Galerkin tensor and
    the table-driven one (SGW_K1_GENERIC=1)."""
    monkeypatch.setenv("SGW_K1_GENERIC", generic)
    prm = workloads.config("cfg2", n=n, xsplits=workloads.uniform_splits(n, ns),
                           ysplits=workloads.uniform_splits(n, ns))
    s = sgw.Solver(prm)
    ref = SGProblem(prm, solver="cg")
    g = torch.Generator().manual_seed(2)
    X = torch.randn(s.P, s.nn, dtype=torch.float64, generator=g)
    Y = s.apply_operator(X.cuda()).cpu().numpy()
    Yo = ref.apply_Kt(X.numpy()[:, ref.mesh.free].T)
    assert rel_l2(Y[:, ref.mesh.free].T, Yo) < 1e-13
    s.close()


def test_single_solve_matches_direct(sgw):
    prm = workloads.config("cfg1")
    s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14)
    s.factor()
    ref = SGProblem(prm)
    g = torch.Generator().manual_seed(3)
    F = torch.zeros(s.P, s.nn, dtype=torch.float64)
    F[:, ref.mesh.free] = torch.randn(s.P, len(ref.mesh.free), dtype=torch.float64, generator=g)
    U, st = s.solve(F.cuda())
    Uo = ref.solve_Kt(F.numpy()[:, ref.mesh.free].T)
    assert rel_l2(U.cpu().numpy()[:, ref.mesh.free].T, Uo) < 1e-10
    assert st["outer_iters"] >= 1
    s.close()


def test_initial_acceleration_matches_oracle(sgw):
    prm = workloads.config("cfg1")
    s = sgw.Solver(prm)
    s.factor()
    s.set_state()
    ref = SGProblem(prm)
    U, V, A = ref.initial_state()
    Ug, Vg, Ag = s.get_state()
    f = ref.mesh.free
    assert rel_l2(Ug.cpu().numpy()[:, f].T, U) < 1e-15
    assert rel_l2(Ag.cpu().numpy()[:, f].T, A) < 1e-12
    assert float(Vg.abs().max()) == 0.0
    s.close()


INNER = [0, 1]  # SGW_INNER_CHOLESKY, SGW_INNER_CHEBYSHEV


@pytest.mark.parametrize("inner", INNER)
def test_cfg1_trajectory_fp64(sgw, inner):
    prm = workloads.config("cfg1")
    (em, es), stats = _trajectory(sgw, prm, 100, 1e-12, inner_prec=inner)
    assert em < 1e-10 and es < 1e-10, (em, es)
    assert all(st["status"] == 0 for st in stats)


@pytest.mark.parametrize("inner", INNER)
def test_uneven_ragged_partition(sgw, inner):
    prm = workloads.config("cfg1", n=37, xsplits=[0, 13, 37], ysplits=[0, 11, 25, 37],
                           x0=0.4, y0=0.6)
    (em, es), _ = _trajectory(sgw, prm, 20, 1e-12, inner_prec=inner)
    assert em < 1e-10 and es < 1e-10, (em, es)


@pytest.mark.parametrize("inner", INNER)
def test_p35_small_mesh(sgw, inner):
    prm = workloads.config("cfg2", n=64, xsplits=workloads.uniform_splits(64, 4),
                           ysplits=workloads.uniform_splits(64, 4), dt=0.004)
    (em, es), _ = _trajectory(sgw, prm, 10, 1e-12, every=5, inner_prec=inner)
    assert em < 1e-10 and es < 1e-10, (em, es)


@pytest.mark.parametrize("deg", [1, 2, 9])
def test_chebyshev_degrees(sgw, deg):
    """Any degree gives an SPD preconditioner: the solution is the same."""
    prm = workloads.config("cfg1")
    (em, es), _ = _trajectory(sgw, prm, 20, 1e-12, inner_prec=1, cheb_degree=deg)
    assert em < 1e-10 and es < 1e-10, (em, es)


def _cheb_tiles(sgw, precision, shape, qs):
    """Set the first feasible q of qs with the given launch shape on both
    subdomain systems (a system the shape cannot cover keeps its tile)."""
    kept = []
    def prep(s):
        for system in (0, 1):
            for q in qs:
                try:
                    s.set_cheb_tile(precision, system, q, shape)
                    kept.append((system, q))
                    break
                except sgw.SGWError:
                    continue
    return prep, kept


@pytest.mark.parametrize("shape", [0, 1, 2])
@pytest.mark.parametrize("ragged", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
def test_chebyshev_launch_shapes(sgw, precision, shape, ragged):
    """Every launch shape of the Chebyshev kernel (1024, 512, 256 threads;
    blocks of 961 and 1089 rows give 1, 2 or 4 rows per thread) with the
    largest feasible mode tile, or a tile that does not divide P = 6."""
    prm = workloads.config("cfg1", n=64, xsplits=workloads.uniform_splits(64, 2),
                           ysplits=workloads.uniform_splits(64, 2))
    qs = [4, 5, 1] if ragged else [8, 7, 6, 5, 4, 3, 2, 1]
    prep, kept = _cheb_tiles(sgw, precision, shape, qs)
    if precision == 0:
        (em, es), _ = _trajectory(sgw, prm, 10, 1e-12, every=5, prep=prep, inner_prec=1)
        assert em < 1e-10 and es < 1e-10, (em, es)
    else:
        (em, es), _ = _trajectory(sgw, prm, 10, 1e-10, every=5, prep=prep, inner_prec=1,
                                  precision=sgw.SGW_FP32_IR64)
        assert em < 1e-6 and es < 1e-6, (em, es)
    assert kept and kept[0][0] == 0, kept  # the Dirichlet system took the shape


def test_sigma_zero_modes_stay_zero(sgw):
    prm = workloads.config("cfg1", sigma=0.0)
    s = sgw.Solver(prm, rtol=1e-12, inner_rtol=1e-14)
    s.factor()
    s.set_state()
    s.step(10)
    U, _, _ = s.get_state()
    assert float(U[1:].abs().max()) == 0.0
    ref = SGProblem(dict(prm, L=0, p_in=0, p_out=0))
    u, v, a = ref.initial_state()
    for _ in range(10):
        u, v, a = ref.step(u, v, a)
    assert rel_l2(U[0].cpu().numpy()[ref.mesh.free], u[:, 0]) < 1e-10
    s.close()


def test_step_before_factor_is_a_state_error(sgw):
    s = sgw.Solver(workloads.config("cfg1"))
    with pytest.raises(sgw.SGWError, match="SGW_ESTATE"):
        s.step(1)
    s.close()


def test_max_iter_one_reports_not_converged(sgw):
    s = sgw.Solver(workloads.config("cfg1"), rtol=1e-12, max_iter=1)
    s.factor()
    s.set_state()
    st = s.step(1)
    assert st["status"] == sgw.SGW_NOT_CONVERGED
    s.close()


def test_resume_from_state_is_bitwise(sgw):
    prm = workloads.config("cfg1")
    a = sgw.Solver(prm, rtol=1e-10)
    a.factor()
    a.set_state()
    a.step(5)
    U, V, A = a.get_state()
    a.step(5)
    ua = a.get_state()[0].clone()
    b = sgw.Solver(prm, rtol=1e-10)
    b.factor()
    b.set_state(U, V, A, step=5)
    b.step(5)
    ub = b.get_state()[0]
    assert torch.equal(ua, ub)
    a.close()
    b.close()


def test_resume_refinement_path_with_carried_images(sgw):
    """Refinement path with stiffness damping: a step takes the damping share
    of the force, K~ Uc, from the images K~ U, K~ V, K~ A carried along with
    the state (the first step after set_state forms them by SG applies).  A
    run resumed from a mid-run state (images formed afresh) and the continued
    run (images carried) agree to far below the refinement tolerance."""
    prm = workloads.config("cfg1")
    kw = dict(rtol=1e-10, precision=sgw.SGW_FP32_IR64)
    a = sgw.Solver(prm, **kw)
    a.factor()
    a.set_state()
    assert a.step(5)["status"] == 0
    U, V, A = [x.clone() for x in a.get_state()]
    assert a.step(5)["status"] == 0
    ua = a.get_state()[0].clone()
    b = sgw.Solver(prm, **kw)
    b.factor()
    b.set_state(U, V, A, step=5)
    assert b.step(5)["status"] == 0
    ub = b.get_state()[0]
    err = float((ua - ub).norm() / ua.norm())
    assert err < 1e-8, err
    a.close()
    b.close()


def test_sg_apply_fp32_kernel(sgw):
    """FP32 operator of the refinement path: relative error ~ FP32 rounding."""
    prm = workloads.config("cfg2", n=64, xsplits=workloads.uniform_splits(64, 4),
                           ysplits=workloads.uniform_splits(64, 4))
    s = sgw.Solver(prm, precision=sgw.SGW_FP32_IR64)
    ref = SGProblem(prm, solver="cg")
    g = torch.Generator().manual_seed(5)
    X = torch.randn(s.P, s.nn, dtype=torch.float64, generator=g)
    Y = s.apply_operator(X.cuda(), precision=sgw.SGW_FP32_IR64).cpu().numpy()
    Yo = ref.apply_Kt(X.numpy()[:, ref.mesh.free].T)
    err = rel_l2(Y[:, ref.mesh.free].T, Yo)
    assert 1e-9 < err < 1e-6, err
    s.close()


@pytest.mark.parametrize("inner", INNER)
@pytest.mark.parametrize("name,over,nsteps,every", [
    ("cfg1", {}, 100, 10),
    ("cfg2", dict(n=64, xsplits=[0, 16, 32, 48, 64], ysplits=[0, 16, 32, 48, 64], dt=0.004), 10, 5),
])
def test_mixed_precision_trajectory(sgw, name, over, nsteps, every, inner):
    """FP32 DD-PCG inside FP64 refinement: the bound 1e-6 on the mean and
    standard deviation (refinement tolerance 1e-10)."""
    prm = workloads.config(name, **over)
    (em, es), stats = _trajectory(sgw, prm, nsteps, 1e-10, every=every,
                                  precision=sgw.SGW_FP32_IR64, inner_prec=inner)
    assert em < 1e-6 and es < 1e-6, (em, es)
    assert all(st["ir_sweeps"] >= st["steps"] for st in stats)


@pytest.mark.parametrize("precision", [0, 1])
def test_graph_replays_give_identical_states(sgw, precision):
    """Inner PCG iterations replayed from captured HIP graphs: the states are
    bitwise those of eager launches (same kernels, same order)."""
    prm = workloads.config("cfg2", n=64, xsplits=workloads.uniform_splits(64, 4),
                           ysplits=workloads.uniform_splits(64, 4), dt=0.004)
    out = []
    for graphs in (False, True):
        s = sgw.Solver(prm, rtol=1e-10, inner_rtol=1e-12, precision=precision, inner_prec=1,
                       cheb_degree=8, graphs=graphs)
        s.factor()
        s.set_state()
        for _ in range(3):
            assert s.step(4)["status"] == 0
        out.append((s.get_state()[0].clone(), s.graph_launches()))
        s.close()
    assert out[0][1] == 0 and out[1][1] > 0
    assert torch.equal(out[0][0], out[1][0])
