"""Pins of the learned-guess network reference (oracle/mlp.py): central
finite differences of the float64 forward pass check the backward pass, and
bfloat16 rounding is checked on values whose rounding is known."""

import numpy as np

from oracle import mlp


def test_bf16_rounding_known_values():
    v = np.array([1.0, 1 + 2**-7, 1 + 2**-8, 1 + 3 * 2**-8, -2.5, 3 * 2**-130])
    r = mlp.round_bf16(v)
    # 1 + 2^-8 is the midpoint of 1 and 1 + 2^-7: ties to the even 1.0;
    # 1 + 3 2^-8 is the midpoint of 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert list(r[:5]) == [1.0, 1 + 2**-7, 1.0, 1 + 2**-6, -2.5]
    assert r[5] == 3 * 2**-130  # subnormal with few bits stays exact


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    ni, ng, H, n = 4, 3, 5, 7
    npar = H * ni + H + H * H + H + ng * H + ng
    w = rng.standard_normal(npar) * 0.5
    x = rng.standard_normal((n, ni))
    t = rng.standard_normal((n, ng))
    loss, g = mlp.loss_grad(w, x, t, ni, ng, H)
    eps = 1e-6
    fd = np.empty(npar)
    for q in range(npar):
        wp, wm = w.copy(), w.copy()
        wp[q] += eps
        wm[q] -= eps
        fd[q] = (mlp.loss_grad(wp, x, t, ni, ng, H)[0]
                 - mlp.loss_grad(wm, x, t, ni, ng, H)[0]) / (2 * eps)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())
    assert np.isclose(loss, np.mean((mlp.forward(w, x, ni, ng, H)[0] - t) ** 2))


def test_layout_and_relu():
    ni, ng, H = 5, 2, 3
    npar = H * ni + H + H * H + H + ng * H + ng
    w = np.zeros(npar)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(w, ni, ng, H)
    assert W1.shape == (H, ni) and W3.shape == (ng, H) and b3.shape == (ng,)
    # only the output bias set: the network returns it for any input
    w[-ng:] = [0.25, -1.5]
    y, _ = mlp.forward(w, np.ones((4, ni)), ni, ng, H)
    assert np.all(y == np.array([0.25, -1.5]))
