"""Newmark average-acceleration time step.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed: Sec. 2, the Newmark update of u and v with
zeta = 1/4, gamma = 1/2; Eq. Kuf / K_T (transient operator
K~ = M/(zeta dt^2) + gamma C/(zeta dt) + K); Eq. fparts, fparts2, UmCm, UmCm2
(effective force f~ = f + M u~_m + C u~_c).  The new acceleration follows by
solving the displacement update for a_{n+1}.
"""


def newmark_step(U, V, A, dt, apply_M, apply_C, solve_Kt, F=None,
                 zeta=0.25, gamma=0.5):
    """One step n -> n+1; returns (U1, V1, A1).

    apply_M / apply_C apply the mass / damping operators, solve_Kt solves
    with the transient operator.  F is the external force at t_{n+1}.
    """
    Um = (U + dt * V) / (zeta * dt * dt) + (1.0 - 2.0 * zeta) * A / (2.0 * zeta)
    Uc = gamma * dt * Um - V - (1.0 - gamma) * dt * A
    Ft = apply_M(Um) + apply_C(Uc)
    if F is not None:
        Ft = Ft + F
    U1 = solve_Kt(Ft, U)
    A1 = U1 / (zeta * dt * dt) - Um
    V1 = V + dt * ((1.0 - gamma) * A + gamma * A1)
    return U1, V1, A1
