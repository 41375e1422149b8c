"""Pins for the oracle's KLE (oracle/kle.py) and log-normal PCE (oracle/lognormal.py).

* The analytic eigenvalues of the exponential kernel are compared with a
  Nystrom discretisation of the integral operator solved by a dense
  symmetric eigensolver (a computation with no shared steps).
* Eigenfunctions are checked for orthonormality and for the integral
  equation itself by quadrature.
* The trace of the covariance operator equals sigma^2 * area, so the sum of
  all eigenvalues approaches sigma^2 from below.
* The log-normal coefficients are compared with Gauss-Hermite projections of
  exp(sum_l g_l xi_l) onto the normalised Hermite basis.
"""

import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He
from scipy.linalg import eigh

from oracle.kle import eval_1d, kle_1d, kle_2d
from oracle.lognormal import lognormal_pce
from oracle.pce import multi_indices


@pytest.mark.parametrize("b", [0.25, 0.3, 0.5, 1.0])
def test_1d_eigenvalues_vs_nystrom(b):
    n = 2000
    x = (np.arange(n) + 0.5) / n            # midpoint rule on [0, 1]
    Kmat = np.exp(-np.abs(x[:, None] - x[None, :]) / b) / n
    ev = np.sort(eigh(Kmat, eigvals_only=True))[::-1][:8]
    modes = kle_1d(b, 8)
    lam = np.array([m[1] for m in modes])
    assert np.all(np.diff(lam) < 0)
    np.testing.assert_allclose(lam, ev, rtol=2e-4)


def test_1d_eigenfunctions_satisfy_integral_equation():
    b = 0.3
    n = 4000
    x = (np.arange(n) + 0.5) / n
    for mode in kle_1d(b, 6):
        phi = eval_1d(mode, x)
        assert abs(np.sum(phi * phi) / n - 1.0) < 1e-6
        for xi in [0.1, 0.37, 0.8]:
            lhs = np.sum(np.exp(-np.abs(xi - x) / b) * phi) / n
            rhs = mode[1] * eval_1d(mode, np.array([xi]))[0]
            assert abs(lhs - rhs) < 1e-5
    ms = kle_1d(b, 6)
    for i in range(6):
        for j in range(i):
            assert abs(np.sum(eval_1d(ms[i], x) * eval_1d(ms[j], x)) / n) < 1e-6


def test_2d_trace_and_order():
    sigma = 0.3
    pairs = kle_2d(sigma, 0.3, 0.3, 200)
    lam = np.array([p[0] for p in pairs])
    assert np.all(np.diff(lam) <= 0)
    assert lam.sum() < sigma ** 2
    assert lam.sum() > 0.9 * sigma ** 2
    # equal correlation lengths: exact tie lambda_12 == lambda_21, (1,2) first
    first = [(p[3], p[4]) for p in kle_2d(0.2, 0.5, 0.5, 3)]
    assert first == [(1, 1), (1, 2), (2, 1)]
    t = kle_2d(0.2, 0.5, 0.5, 3)
    assert t[1][0] == t[2][0]


def test_lognormal_coefficients_vs_quadrature():
    rng = np.random.default_rng(7)
    L, pin = 2, 3
    g = rng.normal(scale=0.3, size=(L, 5))
    kappa = lognormal_pce(g, pin)
    x, w = He.hermegauss(30)
    w = w / math.sqrt(2 * math.pi)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w)

    def he(k, t):
        c = np.zeros(k + 1)
        c[k] = 1.0
        return He.hermeval(t, c)

    for e in range(g.shape[1]):
        field = np.exp(g[0, e] * X1 + g[1, e] * X2)
        assert abs(np.sum(W * field) - kappa[0, e]) < 1e-12
        for k, a in enumerate(multi_indices(L, pin)):
            psi = (he(a[0], X1) * he(a[1], X2)
                   / math.sqrt(math.factorial(a[0]) * math.factorial(a[1])))
            assert abs(np.sum(W * field * psi) - kappa[k, e]) < 1e-12


def test_lognormal_variance_series():
    # sum_{alpha != 0} kappa_alpha^2 -> c0^2 (exp(sum g^2) - 1) as p -> inf
    g = np.array([[0.2], [0.1]])
    kappa = lognormal_pce(g, 12)
    c0 = kappa[0, 0]
    var = np.sum(kappa[1:, 0] ** 2)
    assert abs(var - c0 ** 2 * (math.exp(0.05) - 1.0)) < 1e-14


# ---------------------------------------------------------------------------
# The 2-D field synthesis g_l = sqrt(lambda_l) phi_l^x(x) phi_l^y(y) of
# kle_fields (Sec. 4, Eq. KLEchapt2) against the covariance it must expand
# (Eq. CovarKer2D_chapt2): by Mercer's theorem sum_l g_l(p) g_l(p') converges
# to sigma^2 exp(-|x - x'|/b_x - |y - y'|/b_y) as L grows.  The kernel is
# anisotropic (b_x != b_y) and the point pairs have |dx| far from |dy|, so an
# x/y swap of the eigenfunctions or of the correlation lengths fails, and
# lambda in place of sqrt(lambda) fails by orders of magnitude.
# ---------------------------------------------------------------------------
_KSIG, _KBX, _KBY = 0.3, 0.2, 0.6


def _kle_pairs():
    rng = np.random.Generator(np.random.PCG64(11))
    p = rng.uniform(0.05, 0.95, size=(12, 2))
    d = np.stack([rng.uniform(0.05, 0.3, 12), rng.uniform(0.0, 0.03, 12)], axis=1)
    d[::2] = d[::2, ::-1]  # half the pairs apart along x, half along y
    q = np.clip(p + d * np.where(rng.uniform(size=(12, 1)) < 0.5, -1, 1), 0.0, 1.0)
    return p, q


def _mercer_error(fields, L):
    from oracle.kle import kle_fields
    p, q = _kle_pairs()
    fields = fields or kle_fields
    gp = fields(_KSIG, _KBX, _KBY, L, p[:, 0], p[:, 1])
    gq = fields(_KSIG, _KBX, _KBY, L, q[:, 0], q[:, 1])
    approx = np.sum(gp * gq, axis=0)
    exact = _KSIG ** 2 * np.exp(-np.abs(p[:, 0] - q[:, 0]) / _KBX
                                - np.abs(p[:, 1] - q[:, 1]) / _KBY)
    return np.max(np.abs(approx - exact)) / _KSIG ** 2


def test_kle_fields_converge_to_covariance():
    errs = [_mercer_error(None, L) for L in (50, 200, 800)]
    # the truncation error of the exponential kernel's expansion decays
    # slowly (its eigenvalues fall like 1/w^2); measured 3.0e-2, 8.5e-3,
    # 2.1e-3 of sigma^2 at L = 50, 200, 800
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[1] < 0.015 and errs[2] < 0.004, errs


def _fields_lambda_not_sqrt(sigma, bx, by, L, x, y):
    from oracle.kle import eval_1d, kle_2d
    g = np.zeros((L, len(x)))
    for l, (lam, mx, my, _, _) in enumerate(kle_2d(sigma, bx, by, L)):
        g[l] = lam * eval_1d(mx, x) * eval_1d(my, y)
    return g


def _fields_xy_swapped(sigma, bx, by, L, x, y):
    from oracle.kle import kle_fields
    return kle_fields(sigma, bx, by, L, y, x)


def _fields_lengths_swapped(sigma, bx, by, L, x, y):
    from oracle.kle import kle_fields
    return kle_fields(sigma, by, bx, L, x, y)


@pytest.mark.parametrize("mutant", [_fields_lambda_not_sqrt, _fields_xy_swapped,
                                    _fields_lengths_swapped])
def test_kle_covariance_pin_catches_planted_mistakes(mutant):
    # the same pin applied to plausible mistakes in the synthesis must fail
    assert _mercer_error(mutant, 800) > 0.1
