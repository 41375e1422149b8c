"""Pins for the oracle's polynomial-chaos tensors (oracle/pce.py).

The closed form for E[He_a He_b He_c] is checked against Gauss-Hermite
quadrature (exact for polynomials of degree <= 2n-1), a computation that
shares nothing with the closed form.  Basis sizes are checked against the
numbers the paper prints for its random-variable and order sweeps.
"""

import math

import numpy as np
import pytest
from numpy.polynomial import hermite_e as He

from oracle.pce import galerkin_tensor, he_triple, multi_indices, pce_size


def _gh(n=40):
    x, w = He.hermegauss(n)
    return x, w / math.sqrt(2 * math.pi)


def _he(k, x):
    c = np.zeros(k + 1)
    c[k] = 1.0
    return He.hermeval(x, c)


def test_basis_sizes_match_paper():
    # Sec. 6: 3 RVs order 3 -> 20 terms, 7 RVs order 3 -> 120 terms,
    # 9 RVs order 3 -> 220 terms, 3 RVs order 9 -> 220 terms.
    assert pce_size(3, 3) == 20
    assert pce_size(7, 3) == 120
    assert pce_size(9, 3) == 220
    assert pce_size(3, 9) == 220
    for L, p in [(2, 2), (4, 3), (6, 3), (8, 3), (3, 3)]:
        assert len(multi_indices(L, p)) == pce_size(L, p)
    # Sec. 6: 13,472 vertices x 120 terms ~ 1.6 million unknowns,
    # 37,267 vertices x 220 terms ~ 8.19 million.
    assert round(13472 * pce_size(7, 3) / 1e5) == 16
    assert int(37267 * pce_size(9, 3) / 1e4) == 819


def test_multi_index_order():
    assert multi_indices(2, 2) == [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    mi = multi_indices(3, 3)
    degs = [sum(a) for a in mi]
    assert degs == sorted(degs)
    assert len(set(mi)) == len(mi)


def test_spot_values():
    assert he_triple(2, 2, 2) == 8.0
    assert he_triple(1, 1, 0) == 1.0
    assert he_triple(1, 1, 1) == 0.0
    assert he_triple(0, 0, 0) == 1.0
    assert he_triple(3, 2, 1) == 6.0


def test_triple_closed_form_vs_quadrature():
    x, w = _gh(40)
    for a in range(7):
        for b in range(7):
            for c in range(7):
                q = np.sum(w * _he(a, x) * _he(b, x) * _he(c, x))
                ref = he_triple(a, b, c)
                assert abs(q - ref) <= 1e-9 * max(1.0, abs(ref)), (a, b, c, q, ref)


@pytest.mark.parametrize("L,pin,pout", [(2, 2, 2), (2, 2, 3), (3, 2, 3)])
def test_galerkin_tensor_vs_tensor_quadrature(L, pin, pout):
    c = galerkin_tensor(L, pin, pout)
    x, w = _gh(12)
    grids = np.meshgrid(*([x] * L), indexing="ij")
    wts = np.ones_like(grids[0])
    for d in range(L):
        wts = wts * np.meshgrid(*([w] * L), indexing="ij")[d]

    def psi(alpha):
        v = np.ones_like(grids[0])
        for d, a in enumerate(alpha):
            v = v * _he(a, grids[d]) / math.sqrt(math.factorial(a))
        return v

    kin = multi_indices(L, pin)
    out = multi_indices(L, pout)
    ps = [psi(a) for a in out]
    for k, ak in enumerate(kin):
        pk = psi(ak)
        for i in range(len(out)):
            for j in range(len(out)):
                q = np.sum(wts * pk * ps[i] * ps[j])
                assert abs(q - c[k, i, j]) < 1e-11, (k, i, j, q, c[k, i, j])


def test_tensor_symmetry_and_identity():
    c = galerkin_tensor(4, 2, 3)
    P = c.shape[1]
    np.testing.assert_array_equal(c[0], np.eye(P))          # G_0 = I (normalised)
    np.testing.assert_array_equal(c, np.transpose(c, (0, 2, 1)))
    # <psi_k psi_i psi_0> = delta_ki for k in the input basis
    for k in range(c.shape[0]):
        e = np.zeros(P)
        e[k] = 1.0
        np.testing.assert_array_equal(c[k, :, 0], e)
