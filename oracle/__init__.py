"""CPU FP64 oracle for the stochastic Galerkin acoustic-wave solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the C-ABI library,
its HIP kernels or its Python binding) may import, call or link anything in
this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

What it computes is the plain definition of one Newmark time step of the
stochastic Galerkin (SG) system, with no domain decomposition at all:

* P1 finite elements on a structured triangle mesh of the unit square
  (weak form and semi-discretisation, Sec. 2, Eq. acoustic_ode);
* the log-normal squared wave speed c_s = exp(g) with g a Karhunen-Loeve
  expansion of an exponential-covariance Gaussian field
  (Sec. 4, Eq. CovarKer2D_chapt2, KLEchapt2, c0pce, LNL0);
* normalised Hermite polynomial chaos and its Galerkin projection
  (Eq. PCEOrtho, galerproject_chap2, stok, sto_masschap2), Rayleigh damping
  with deterministic mass (Appendix, Rayleigh damping);
* Newmark average-acceleration stepping (Sec. 2, Eq. K_T, Kuf, fparts,
  UmCm) of the SG system (Eq. K_T_Sto), each step solved directly
  (sparse LU of the SG matrix) or by CG preconditioned with the
  mean-matrix factor to a relative residual of 1e-14.

Everything is float64.  Every function cites the passage it follows.
Pins that tie this code to the paper and to mathematics live in
``tests/test_oracle_*.py``.  Parity unpinned: none (every function has a pin).
"""

from .pce import multi_indices, pce_size, he_triple, galerkin_tensor  # noqa: F401
from .kle import kle_1d, kle_2d  # noqa: F401
from .lognormal import lognormal_pce  # noqa: F401
from .fem import StructuredMesh, assemble  # noqa: F401
from .sg import SGProblem  # noqa: F401
from .newmark import newmark_step  # noqa: F401
