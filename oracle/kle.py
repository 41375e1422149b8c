"""Karhunen-Loeve expansion of the separable exponential covariance.

Test infrastructure only (see ``oracle/__init__.py``).

Paper passages followed: Sec. 4, Eq. CovarKer2D_chapt2 (covariance
sigma^2 exp(-(|x1-x2|/b_x + |y1-y2|/b_y))) and Eq. KLEchapt2
(g = g_0 + sum_{n<=L} xi_n sqrt(lambda_n) phi_n).  The paper does not say how
the eigenpairs are obtained; the reading used is the classical closed form
for the exponential kernel on an interval [-a, a] (here a = 1/2 after shifting
[0, 1]), with c = 1/b:

* even modes: c - w tan(w a) = 0,  phi = cos(w x) / sqrt(a + sin(2 w a)/(2 w))
* odd modes:  w + c tan(w a) = 0,  phi = sin(w x) / sqrt(a - sin(2 w a)/(2 w))
* eigenvalue: lambda = 2 c / (w^2 + c^2)   (unit variance).

The 2-D kernel is a product of two 1-D kernels, so its eigenpairs are the
products sigma^2 lambda_m^x lambda_n^y, phi_m^x(x) phi_n^y(y).  They are
sorted by decreasing eigenvalue, ties broken by (m, n) ascending, and the
first L are kept.  The 1-D product is formed first so that swapped pairs
(m, n), (n, m) of an isotropic kernel tie exactly.
"""

import math

import numpy as np
from scipy.optimize import brentq


def kle_1d(b, nmodes, a=0.5):
    """First ``nmodes`` 1-D eigenpairs of exp(-|x-y|/b) on [-a, a].

    Returns a list of (omega, lam, parity) with parity 0 = even (cos) and
    1 = odd (sin), in order of increasing omega (= decreasing lam).  The
    roots are bracketed where the transcendental equations change sign:
    even roots lie in (n pi/a, n pi/a + pi/(2a)), odd roots in
    (n pi/a + pi/(2a), (n+1) pi/a).
    """
    c = 1.0 / b
    modes = []
    n = 0
    while len(modes) < nmodes:
        lo, hi = n * math.pi / a, n * math.pi / a + math.pi / (2 * a)
        # even: c cos(w a) - w sin(w a) = 0   (tan form multiplied by cos)
        w = brentq(lambda w: c * math.cos(w * a) - w * math.sin(w * a),
                   lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        modes.append((w, 2 * c / (w * w + c * c), 0))
        if len(modes) == nmodes:
            break
        lo, hi = hi, (n + 1) * math.pi / a
        # odd: w cos(w a) + c sin(w a) = 0
        w = brentq(lambda w: w * math.cos(w * a) + c * math.sin(w * a),
                   lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        modes.append((w, 2 * c / (w * w + c * c), 1))
        n += 1
    return modes


def eval_1d(mode, x, a=0.5):
    """Normalised 1-D eigenfunction at points x of [0, 1] (shifted by a)."""
    w, _, parity = mode
    t = np.asarray(x, dtype=np.float64) - a
    if parity == 0:
        return np.cos(w * t) / math.sqrt(a + math.sin(2 * w * a) / (2 * w))
    return np.sin(w * t) / math.sqrt(a - math.sin(2 * w * a) / (2 * w))


def kle_2d(sigma, bx, by, L):
    """The L dominant 2-D eigenpairs as (lam, mode_x, mode_y, m, n).

    m, n are 1-based 1-D mode numbers; lam includes sigma^2.
    """
    nper = L + 2
    mx = kle_1d(bx, nper)
    my = kle_1d(by, nper)
    cand = []
    for m in range(nper):
        for n in range(nper):
            lam = sigma * sigma * (mx[m][1] * my[n][1])
            cand.append((-lam, m + 1, n + 1))
    cand.sort()
    out = []
    for neg, m, n in cand[:L]:
        out.append((-neg, mx[m - 1], my[n - 1], m, n))
    return out


def kle_fields(sigma, bx, by, L, x, y):
    """g_l(x, y) = sqrt(lam_l) phi_l(x, y), shape (L, len(x)); g_0 = 0."""
    pairs = kle_2d(sigma, bx, by, L)
    g = np.zeros((L, len(x)))
    for l, (lam, modx, mody, _, _) in enumerate(pairs):
        g[l] = math.sqrt(lam) * eval_1d(modx, x) * eval_1d(mody, y)
    return g
