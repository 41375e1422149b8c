"""Host-side tables and host logic of the HIP path, without a GPU.

The generated SG-apply kernels carry the Galerkin tensor
c_kij = <psi_k psi_i psi_j> (Eq. galerproject_chap2 with the normalised
Hermite basis of Eq. PCEOrtho) as immediates, listed by the generator in the
chaos order of the solver's coefficient and solution arrays.  Every basis the
library generates code for is compared entry by entry with the oracle's dense
tensor: the same multi-index order, the same nonzero pattern, the same values.
The roofline accounting of bench.py (bytes and flops per row of one SG
apply) is checked against counts taken from the oracle's tensor, and its
refusal of more than one GPU.
"""

import numpy as np
import pytest

import bench
import workloads
from oracle.pce import galerkin_tensor, pce_size
from paper_2512_23027_amd import gen_k1

BASES = sorted(gen_k1.BASES)


@pytest.mark.parametrize("L,p_in,p_out", BASES)
def test_generated_tensor_matches_oracle(L, p_in, p_out):
    nk, P, ent = gen_k1.entries(L, p_in, p_out)
    assert nk == pce_size(L, p_in) and P == pce_size(L, p_out)
    # no random variable (the deterministic medium): one mode, psi_0 = 1, and
    # the triple product is the empty product 1
    c = galerkin_tensor(L, p_in, p_out) if L > 0 else np.ones((1, 1, 1))
    mine = np.zeros_like(c)
    for k, i, j, v in ent:
        assert mine[k, i, j] == 0.0  # each entry listed once
        mine[k, i, j] = v
    np.testing.assert_array_equal(mine != 0.0, np.abs(c) > 1e-14)
    np.testing.assert_allclose(mine, c, rtol=1e-13, atol=0.0)


def test_bench_counts_follow_the_oracle_tensor():
    """Bytes per row 7 (M+1) 4 + 7 * 4 + 2 P 4, flops per row
    2 (7 |KJ| + nnz(c)) for the 512x512 workload's basis (L = 8, P = 165)."""
    prm = workloads.config("cfg5")
    c = galerkin_tensor(prm["L"], prm["p_in"], prm["p_out"])
    nz = np.abs(c) > 1e-14
    nk, P = c.shape[0], c.shape[1]
    kj = int(nz.any(axis=1).sum())  # distinct (k, j) pairs with an entry
    bpr, fpr, fused = bench.sg_apply_counts(prm)
    assert bpr == 7 * nk * 4 + 7 * 4 + 2 * P * 4
    assert fpr == 2 * (7 * kj + int(nz.sum()))
    assert fused == 2 * P * 4
    assert (nk, P, kj, int(nz.sum())) == (45, 165, 3701, 4413)


SHARED = [(b, T) for b in sorted(gen_k1.SHARED) for T in sorted(gen_k1.SHARED[b])]


@pytest.mark.parametrize("basis,T", SHARED)
def test_shared_kernel_plan_covers_every_product_once(basis, T):
    """Work plan of the shared-halo SG-apply kernels: over the output groups,
    every coefficient matrix with products on a group's outputs is owned by
    exactly one wave in sub-chunks of at most KC matrices; the greedy deal
    leaves the waves' loads within one matrix's work of each other; the
    reduction slices cover the group within the LDS budget; the groups
    cover every output mode once."""
    L, p_in, p_out = basis
    cfg = gen_k1.shared_cfg(L, p_in, p_out, T)
    nk, P, ent = gen_k1.entries(L, p_in, p_out)
    w = 4 if T == "float" else 8
    groups = gen_k1.shared_groups(L, p_in, p_out, T)
    assert groups[0][0] == 0 and groups[-1][1] == P
    assert all(a[1] == b[0] for a, b in zip(groups, groups[1:]))
    for i0, i1 in groups:
        NW, MT, waves, R, sl = gen_k1.shared_plan(L, p_in, p_out, T, i0, i1)
        cost = {}
        pairs = {}
        for k, i, j, _ in ent:
            if i0 <= i < i1:
                pairs.setdefault(k, set()).add(j)
                cost[k] = cost.get(k, 0) + 1
        cost = {k: cost[k] + 7 * len(pairs[k]) for k in cost}
        owned = [k for wave in waves for chunk in wave for k in chunk]
        assert sorted(owned) == sorted(cost)  # each matrix with work, once
        assert all(len(chunk) <= cfg["KC"] for wave in waves for chunk in wave)
        loads = [sum(cost[k] for chunk in wave for k in chunk) for wave in waves]
        assert len(waves) == NW
        assert max(loads) - min(loads) <= max(cost.values())
        assert R * sl >= i1 - i0 and (R - 1) * sl < i1 - i0
        assert NW * sl * 64 * w <= cfg["RB"] or R == i1 - i0
        assert MT == min(cfg["MT"], P)


def test_bench_refuses_several_gpus():
    """bench.py measures one GPU: --gpus above 1 ends with a message and exit
    status 2 before touching a device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
