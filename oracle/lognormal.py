"""Polynomial-chaos coefficients of the log-normal squared wave speed.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed: Sec. 4, Eq. c0pce and Eq. LNL0.  c_s = exp(g) with
g = g_0 + sum_l g_l(x) xi_l; its mean is c_0 = exp(g_0 + 1/2 sum_l g_l^2).
The printed coefficient formula is garbled in the available text (it speaks of
expectations of functionals centred at g_i); the reading used is the standard
projection onto the normalised Hermite basis:

    kappa_alpha(x) = <exp(g) psi_alpha> = c_0(x) prod_d g_d(x)^alpha_d / sqrt(alpha_d!)

which equals c_0 <psi_alpha(xi + g)>, i.e. the expectation of the basis
functional centred at g.
"""

import math

import numpy as np

from .pce import multi_indices


def lognormal_pce(g, p_in, g0=0.0):
    """kappa[k, e] for the input basis |alpha| <= p_in.

    g has shape (L, ne): the KLE fields at the evaluation points.
    """
    L, ne = g.shape
    c0 = np.exp(g0 + 0.5 * np.sum(g * g, axis=0))
    idx = multi_indices(L, p_in)
    kappa = np.zeros((len(idx), ne))
    for k, alpha in enumerate(idx):
        v = c0.copy()
        for d in range(L):
            if alpha[d]:
                v = v * g[d] ** alpha[d] / math.sqrt(math.factorial(alpha[d]))
        kappa[k] = v
    return kappa
