"""The stochastic Galerkin wave system and its time stepping, without DD.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed:
* Eq. galerproject_chap2, sto_masschap2, stok: [K]_{jk} = sum_i G_ijk K_i and
  the block-diagonal deterministic mass <psi_j psi_k> delta_jk M (normalised
  basis, so the SG mass is I_P (x) M);
* Appendix, Rayleigh damping: C_0 = alpha0 M + alpha1 K_0, C_k = alpha1 K_k;
* Eq. K_T_Sto: SG transient operator M/(zeta dt^2) + gamma C/(zeta dt) + K;
* Sec. 2 Newmark stepping (``newmark.py``); Alg. 1 supplies u_0, v_0, a_0
  and the paper's pulse initial condition (Eq. initial_2Dwave).

Each step solves K~ U_{n+1} = F~ either directly (sparse LU of the assembled
SG matrix, factored once since K~ does not change in time) or by conjugate
gradients preconditioned with I_P (x) K~_0^{-1} to a relative residual of
1e-14.  The readings for a_0 (solved from M a_0 = f_0 - C v_0 - K u_0), the
pulse width (alpha = width^2) and the output moments (mean = mode 0,
variance = sum of squares of modes >= 1 in the normalised basis) are
readings of points the paper leaves open.

Vectors are numpy arrays of shape (N_free, P): row = free node, column = PCE
mode.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import StructuredMesh, assemble
from .kle import kle_fields
from .lognormal import lognormal_pce
from .newmark import newmark_step
from .pce import galerkin_tensor


class SGProblem:
    """One stochastic wave problem (all parameters in a plain dict).

    Keys: n, L, sigma, bx, by, p_in, p_out, dt, alpha0, alpha1, and the
    initial pulse x0, y0, width, amp (or ``u0``, an array over all mesh
    nodes).  Optional: zeta (1/4), gamma (1/2).
    """

    def __init__(self, prm, solver="direct"):
        self.prm = dict(prm)
        self.zeta = prm.get("zeta", 0.25)
        self.gamma = prm.get("gamma", 0.5)
        self.dt = prm["dt"]
        self.mesh = mesh = StructuredMesh(prm["n"])
        L = prm["L"]
        if L > 0:
            g = kle_fields(prm["sigma"], prm["bx"], prm["by"], L,
                           mesh.cx, mesh.cy)
        else:
            g = np.zeros((0, len(mesh.cx)))
        self.kappa = lognormal_pce(g, prm["p_in"]) if L > 0 else \
            np.ones((1, len(mesh.cx)))
        self.c = galerkin_tensor(L, prm["p_in"], prm["p_out"]) if L > 0 \
            else np.ones((1, 1, 1))
        self.nk, self.P = self.c.shape[0], self.c.shape[1]
        Kall, Mall = assemble(mesh, self.kappa)
        f = mesh.free
        self.K = [Kk[f][:, f].tocsr() for Kk in Kall]
        self.M = Mall[f][:, f].tocsr()
        a0, a1 = prm.get("alpha0", 0.0), prm.get("alpha1", 0.0)
        self.alpha0, self.alpha1 = a0, a1
        z, gm, dt = self.zeta, self.gamma, self.dt
        # K~_k of Eq. K_T_Sto with C_0 = a0 M + a1 K_0, C_k = a1 K_k
        self.Kt = []
        for k in range(self.nk):
            Ck = a1 * self.K[k] + (a0 * self.M if k == 0 else 0 * self.M)
            Mk = self.M if k == 0 else 0 * self.M
            self.Kt.append((Mk / (z * dt * dt) + gm * Ck / (z * dt)
                            + self.K[k]).tocsr())
        self.N = len(f)
        self._lu = None
        self._mlu = None
        self._k0lu = None
        self.solver = solver
        self.cg_iters = []

    # -- SG operators on (N, P) arrays ------------------------------------
    def _sg_apply(self, mats, U):
        """Y[:, i] = sum_k sum_j c[k, i, j] mats[k] U[:, j]."""
        Y = np.zeros_like(U)
        for k in range(self.nk):
            Y += (mats[k] @ U) @ self.c[k].T
        return Y

    def apply_K(self, U):
        return self._sg_apply(self.K, U)

    def apply_M(self, U):
        return self.M @ U

    def apply_C(self, U):
        return self.alpha0 * (self.M @ U) + self.alpha1 * self.apply_K(U)

    def apply_Kt(self, U):
        return self._sg_apply(self.Kt, U)

    def assembled_Kt(self):
        """The SG transient matrix, node-major (row n*P + i)."""
        A = None
        for k in range(self.nk):
            t = sp.kron(self.Kt[k], sp.csr_matrix(self.c[k]), format="csr")
            A = t if A is None else A + t
        return A.tocsc()

    # -- solves -------------------------------------------------------------
    def solve_Kt(self, F, U_prev=None):
        if self.solver == "direct":
            if self._lu is None:
                self._lu = spla.splu(self.assembled_Kt())
            return self._lu.solve(F.reshape(-1)).reshape(F.shape)
        return self._solve_cg(F, U_prev)

    def _solve_cg(self, F, X0, rtol=1e-14, maxit=500):
        """CG with the mean preconditioner I_P (x) K~_0^{-1}."""
        if self._k0lu is None:
            self._k0lu = spla.splu(self.Kt[0].tocsc())
        X = np.zeros_like(F) if X0 is None else X0.copy()
        R = F - self.apply_Kt(X)
        bnorm = np.linalg.norm(F)
        if bnorm == 0.0:
            self.cg_iters.append(0)
            return np.zeros_like(F)
        Z = self._k0lu.solve(R)
        Pd = Z.copy()
        rz = np.vdot(R, Z)
        for it in range(maxit):
            if np.linalg.norm(R) <= rtol * bnorm:
                self.cg_iters.append(it)
                return X
            Q = self.apply_Kt(Pd)
            alpha = rz / np.vdot(Pd, Q)
            X += alpha * Pd
            R -= alpha * Q
            Z = self._k0lu.solve(R)
            rz_new = np.vdot(R, Z)
            Pd = Z + (rz_new / rz) * Pd
            rz = rz_new
        raise RuntimeError("oracle CG did not reach rtol=%g" % rtol)

    # -- initial state and stepping ------------------------------------------
    def initial_state(self):
        """U_0 (pulse in mode 0), V_0 = 0, A_0 from M A_0 = -K U_0 - C V_0.

        Random initial conditions (Eq. acous_sto: u_0(x, theta) and
        v_0(x, theta)) are given by their chaos coefficients in the output
        basis: ``u0_modes`` / ``v0_modes``, arrays of shape (P, (n+1)^2)
        over all mesh nodes (mode-major), replacing the pulse / zero."""
        prm, mesh = self.prm, self.mesh
        U = np.zeros((self.N, self.P))
        if "u0_modes" in prm:
            U[:] = np.asarray(prm["u0_modes"], dtype=np.float64)[:, mesh.free].T
        elif "u0" in prm:
            U[:, 0] = np.asarray(prm["u0"], dtype=np.float64)[mesh.free]
        else:
            r2 = (mesh.x - prm["x0"]) ** 2 + (mesh.y - prm["y0"]) ** 2
            U[:, 0] = (prm.get("amp", 1.0)
                       * np.exp(-r2 / (prm["width"] ** 2)))[mesh.free]
        V = np.zeros_like(U)
        if "v0_modes" in prm:
            V[:] = np.asarray(prm["v0_modes"], dtype=np.float64)[:, mesh.free].T
        if self._mlu is None:
            self._mlu = spla.splu(self.M.tocsc())
        A = self._mlu.solve(-self.apply_K(U) - self.apply_C(V))
        return U, V, A

    def step(self, U, V, A):
        return newmark_step(U, V, A, self.dt, self.apply_M, self.apply_C,
                            self.solve_Kt, zeta=self.zeta, gamma=self.gamma)

    def moments(self, U):
        """(mean, std) over all (n+1)^2 mesh nodes, zero on the boundary."""
        mean = np.zeros(self.mesh.nn)
        std = np.zeros(self.mesh.nn)
        mean[self.mesh.free] = U[:, 0]
        std[self.mesh.free] = np.sqrt(np.sum(U[:, 1:] ** 2, axis=1))
        return mean, std

    def run(self, nsteps, record=None):
        """Advance nsteps; return {step: (mean, std)} at the recorded steps.

        ``record`` is a set of step numbers (default: every step).
        """
        U, V, A = self.initial_state()
        out = {}
        if record is None or 0 in record:
            out[0] = self.moments(U)
        for s in range(1, nsteps + 1):
            U, V, A = self.step(U, V, A)
            if record is None or s in record:
                out[s] = self.moments(U)
        self.state = (U, V, A)
        return out


def energy(prob, U, V):
    """Discrete energy 1/2 V'(I(x)M)V + 1/2 U'K U of the undamped SG system."""
    return 0.5 * np.vdot(V, prob.apply_M(V)) + 0.5 * np.vdot(U, prob.apply_K(U))


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 (the error measure of Eq. Norm)."""
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


__all__ = ["SGProblem", "energy", "rel_l2", "math"]
