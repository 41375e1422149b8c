"""Plain reference of the learned-guess network (not a method of the paper).

Test infrastructure only (see ``oracle/__init__.py``).

The interface-PCG initial guess may come from a small multilayer perceptron
(an addition of this build; the paper starts from the previous solution,
Alg. 1).  This module is its reference, written independently of the HIP
kernels: numpy, float64 accumulation.  With ``bf16=True`` every operand of a
matrix product is first rounded to bfloat16 (round to nearest even), as the
GPU's matrix cores see them; with ``bf16=False`` it is the exact float64
network, whose backward pass is pinned by central finite differences of its
forward pass (tests/test_oracle_mlp.py).

Network: x (n, n_in) -> h1 = relu(x W1^T + b1) -> h2 = relu(h1 W2^T + b2)
-> y = h2 W3^T + b3 (n, n_out); loss = mean((y - t)^2) over all entries.
Parameter vector layout: [W1 (H x n_in, row-major), b1, W2 (H x H), b2,
W3 (n_out x H), b3].
"""

import numpy as np


def round_bf16(a):
    """float -> bfloat16 -> float, round to nearest even (finite values)."""
    a32 = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def unpack(w, n_in, n_out, hidden):
    """Split the parameter vector into (W1, b1, W2, b2, W3, b3)."""
    w = np.asarray(w, dtype=np.float64)
    ni, H, ng = n_in, hidden, n_out
    sizes = [H * ni, H, H * H, H, ng * H, ng]
    parts, o = [], 0
    for s in sizes:
        parts.append(w[o:o + s])
        o += s
    assert o == w.size
    W1, b1, W2, b2, W3, b3 = parts
    return W1.reshape(H, ni), b1, W2.reshape(H, H), b2, W3.reshape(ng, H), b3


def _mm(a, b, bf16):
    if bf16:
        a, b = round_bf16(a), round_bf16(b)
    return a @ b


def forward(w, x, n_in, n_out, hidden, bf16=False):
    """Outputs y and the hidden activations (h1, h2)."""
    W1, b1, W2, b2, W3, b3 = unpack(w, n_in, n_out, hidden)
    x = np.asarray(x, dtype=np.float64)
    h1 = np.maximum(_mm(x, W1.T, bf16) + b1, 0.0)
    h2 = np.maximum(_mm(h1, W2.T, bf16) + b2, 0.0)
    y = _mm(h2, W3.T, bf16) + b3
    return y, (h1, h2)


def loss_grad(w, x, t, n_in, n_out, hidden, bf16=False):
    """Mean squared error and its gradient in the parameter layout."""
    W1, b1, W2, b2, W3, b3 = unpack(w, n_in, n_out, hidden)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    y, (h1, h2) = forward(w, x, n_in, n_out, hidden, bf16)
    n = y.size
    e = y - t
    loss = float((e * e).sum() / n)
    dy = 2.0 * e / n
    gW3 = _mm(dy.T, h2, bf16)
    gb3 = dy.sum(axis=0)
    d2 = _mm(dy, W3, bf16) * (h2 > 0)
    gW2 = _mm(d2.T, h1, bf16)
    gb2 = d2.sum(axis=0)
    d1 = _mm(d2, W2, bf16) * (h1 > 0)
    gW1 = _mm(d1.T, x, bf16)
    gb1 = d1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g
