"""Seeded synthetic workloads: problem parameters and random input draws.

This module holds no arithmetic of the solver method.  It only names the
workloads (mesh size, random-field parameters, PCE orders, time step,
partition, tolerances) and draws their seeded random inputs (pulse centres,
per-problem random-field parameters and rectilinear subdomain splits) with
numpy's PCG64.  The oracle, the tests and the benchmark all take their
inputs from here.

Defaults that the workload descriptions leave open follow the paper:
Rayleigh damping alpha0 = 0.5445, alpha1 = 0.0174 (Sec. 6.2), pulse
amplitude 1 (Eq. initial_2Dwave), input PCE order 2 (Sec. 6 setup).
"""

import numpy as np

ALPHA0, ALPHA1 = 0.5445, 0.0174


def pulse_centre(seed):
    """Pulse centre drawn from U[0.2, 0.8]^2."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0, y0 = rng.uniform(0.2, 0.8, size=2)
    return float(x0), float(y0)


def uniform_splits(n, ns):
    """Cut positions (in cells) of ns equal strips of an n-cell side."""
    assert n % ns == 0
    return [i * (n // ns) for i in range(ns + 1)]


def random_splits(rng, n, counts=(8, 9, 10), lo=0.71, hi=1.41,
                  area_band=(0.5, 2.0), min_cells=4):
    """Seeded rectilinear splits whose cell areas lie within area_band x mean."""
    while True:
        nx = int(rng.choice(counts))
        ny = int(rng.choice(counts))
        cuts = []
        for m in (nx, ny):
            w = rng.uniform(lo, hi, size=m)
            pos = np.round(np.concatenate([[0.0], np.cumsum(w)]) / w.sum() * n)
            cuts.append([int(p) for p in pos])
        wx = np.diff(cuts[0])
        wy = np.diff(cuts[1])
        if wx.min() < min_cells or wy.min() < min_cells:
            continue
        area = np.outer(wy, wx).astype(np.float64)
        mean = n * n / (nx * ny)
        if area.min() >= area_band[0] * mean and area.max() <= area_band[1] * mean:
            return cuts[0], cuts[1]


def base(n, L, sigma, b, p_out, dt, nsteps, rtol, xs, ys, x0=0.5, y0=0.5,
         p_in=2, width=0.05):
    return dict(n=n, L=L, sigma=sigma, bx=b, by=b, p_in=p_in, p_out=p_out,
                dt=dt, nsteps=nsteps, rtol=rtol, alpha0=ALPHA0, alpha1=ALPHA1,
                x0=x0, y0=y0, width=width, amp=1.0, xsplits=xs, ysplits=ys)


def config(name, **over):
    """Parameter dict of a named workload; keyword overrides are applied last.

    cfg1  32x32 mesh, 2x2 subdomains, L=2, sigma 0.2, b 0.5, order 2 (P=6),
          dt 0.005, 100 steps, pulse at (0.5, 0.5), rtol 1e-10.
    cfg2  256x256 mesh, 8x8 subdomains, L=4, sigma 0.3, b 0.3, order 3
          (P=35), dt 0.001, 500 steps, pulse centre from seed 2, rtol 1e-8.
    cfg5  512x512 mesh, 16x16 subdomains, L=8, sigma 0.3, b 0.25, order 3
          (P=165), dt 0.001, 1000 steps, pulse centre from seed 5, rtol 1e-8.
    cfg3-<p>  problem p (0..7) of the batched set: 384x384 mesh, seeded
          rectilinear splits with 8-10 strips per side (cells within 0.5-2x
          the mean area), sigma ~ U[0.1, 0.4], b ~ U[0.2, 0.6], L=6, order 3
          (P=84), dt 0.001, 500 steps, rtol 1e-8; all draws from seed 300+p.
    """
    if name == "cfg1":
        c = base(32, 2, 0.2, 0.5, 2, 0.005, 100, 1e-10,
                 uniform_splits(32, 2), uniform_splits(32, 2))
    elif name == "cfg2":
        x0, y0 = pulse_centre(2)
        c = base(256, 4, 0.3, 0.3, 3, 0.001, 500, 1e-8,
                 uniform_splits(256, 8), uniform_splits(256, 8), x0, y0)
    elif name == "cfg5":
        x0, y0 = pulse_centre(5)
        c = base(512, 8, 0.3, 0.25, 3, 0.001, 1000, 1e-8,
                 uniform_splits(512, 16), uniform_splits(512, 16), x0, y0)
    elif name.startswith("cfg3-"):
        p = int(name.split("-")[1])
        rng = np.random.Generator(np.random.PCG64(300 + p))
        sigma = float(rng.uniform(0.1, 0.4))
        b = float(rng.uniform(0.2, 0.6))
        xs, ys = random_splits(rng, 384)
        x0, y0 = (float(v) for v in rng.uniform(0.2, 0.8, size=2))
        c = base(384, 6, sigma, b, 3, 0.001, 500, 1e-8, xs, ys, x0, y0)
    else:
        raise KeyError(name)
    c.update(over)
    return c


def learned_guess_seeds():
    """Pulse-centre seeds of the learned-guess study on the cfg1 problem:
    10 training trajectories of 200 steps, 5 held-out locations."""
    return list(range(400, 410)), list(range(500, 505))


def cfg4(seed, **over):
    """The cfg1 problem with its pulse centre drawn from ``seed``."""
    x0, y0 = pulse_centre(seed)
    over.setdefault("nsteps", 200)
    return config("cfg1", x0=x0, y0=y0, **over)
