"""Hermite polynomial chaos: multi-indices and Galerkin triple products.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed:
* Eq. PCEOrtho and the statement in the numerical-results setup that the PCE
  basis is normalised: psi_alpha = prod_d He_{alpha_d}(xi_d) / sqrt(alpha_d!),
  so <psi_i psi_j> = delta_ij.
* Eq. galerproject_chap2 / stok: G_ijk = <psi_i psi_j psi_k>.
* Sec. 6 (scalability in random variables and order): the number of terms of
  a total-degree basis in L variables of order p is (L+p)!/(L! p!).

The multi-index order is not stated in the paper; the reading used is graded
by total degree, then descending lexicographic inside one degree, e.g. for
L=2: (0,0), (1,0), (0,1), (2,0), (1,1), (0,2).
"""

import itertools
import math

import numpy as np


def pce_size(L, p):
    """Number of total-degree Hermite chaos terms, (L+p)!/(L! p!)."""
    return math.comb(L + p, p)


def multi_indices(L, p):
    """All alpha in N^L with |alpha| <= p, graded then descending-lex."""
    out = []
    for deg in range(p + 1):
        level = [a for a in itertools.product(range(deg + 1), repeat=L)
                 if sum(a) == deg]
        level.sort(reverse=True)
        out.extend(level)
    return out


def he_triple(a, b, c):
    """E[He_a He_b He_c] for xi ~ N(0,1), probabilists' Hermite polynomials.

    Closed form: with a+b+c = 2s even and s >= max(a,b,c) the expectation is
    a! b! c! / ((s-a)! (s-b)! (s-c)!); otherwise it is zero.
    """
    tot = a + b + c
    if tot % 2:
        return 0.0
    s = tot // 2
    if s < a or s < b or s < c:
        return 0.0
    return float(math.factorial(a) * math.factorial(b) * math.factorial(c)
                 // (math.factorial(s - a) * math.factorial(s - b)
                     * math.factorial(s - c)))


def galerkin_tensor(L, p_in, p_out):
    """Dense c[k, i, j] = <psi_k psi_i psi_j> (normalised basis).

    k runs over the input (coefficient) basis |alpha| <= p_in, i and j over
    the output basis |alpha| <= p_out.  The expectation factorises over the
    independent xi_d, so it is the product over dimensions of the 1-D
    normalised triple products (Eq. galerproject_chap2 with Eq. PCEOrtho).
    """
    kin = np.array(multi_indices(L, p_in), dtype=np.int64).reshape(-1, L)
    out = np.array(multi_indices(L, p_out), dtype=np.int64).reshape(-1, L)
    n = max(p_in, p_out) + 1
    e1 = np.zeros((n, n, n))
    for a in range(n):
        for b in range(n):
            for cc in range(n):
                e1[a, b, cc] = he_triple(a, b, cc) / math.sqrt(
                    math.factorial(a) * math.factorial(b) * math.factorial(cc))
    c = np.ones((len(kin), len(out), len(out)))
    for d in range(L):
        c *= e1[kin[:, d][:, None, None], out[:, d][None, :, None],
                out[:, d][None, None, :]]
    return c
