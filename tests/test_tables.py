"""Host-side tables of the HIP path against the oracle, without a GPU.

The generated SG-apply kernels carry the Galerkin tensor
c_kij = <psi_k psi_i psi_j> (Eq. galerproject_chap2 with the normalised
Hermite basis of Eq. PCEOrtho) as immediates, listed by the generator in the
chaos order of the solver's coefficient and solution arrays.  Every basis the
library generates code for is compared entry by entry with the oracle's dense
tensor: the same multi-index order, the same nonzero pattern, the same values.
The roofline accounting of bench.py (bytes and flops per row of one SG
apply) is checked against counts taken from the oracle's tensor.
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
