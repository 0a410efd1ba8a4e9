"""The library's multigrid setup (host code, no device) against the oracle's: the finest
level's aggregates are equal node for node, the level sizes are equal, and the stored
entries per level agree (both drop entries that sum to exactly zero; a rounding
difference could only change that count marginally)."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg, sparse, walks


def cases():
    out = []
    rp, ci = synth.road_grid(60, 60, 0.7, seed=7)
    out.append(("grid", len(rp) - 1, rp, ci, 1.0, 0.99))
    out.append(("grid", len(rp) - 1, rp, ci, 0.5, 0.3162))
    rp, ci = synth.barabasi_albert(3000, 5, 3)
    out.append(("ba", 3000, rp, ci, 1.0, 0.9))
    out.append(("ba", 3000, rp, ci, 0.0, 0.001))
    rp, ci = synth.stochastic_block_model(2000, 8, 10, 20, 5)
    out.append(("sbm", 2000, rp, ci, 0.25, 0.9))
    return out


@pytest.mark.parametrize("case", range(5))
def test_hierarchy_matches_oracle(lib, case):
    name, n, rp, ci, mu, frac = cases()[case]
    Adj = sparse.adjacency(n, rp, ci)
    alpha = frac / sparse.rho_Z(Adj, mu)
    rows, nnz, agg = lib.amg_describe(n, rp, ci, mu, alpha)
    A = sp.csr_matrix(sparse.deformed(Adj, mu, alpha))
    A.eliminate_zeros()
    ref_agg, _ = amg.vmb_aggregate(A, 0.01)
    levels = amg.hierarchy(A)
    np.testing.assert_array_equal(agg, ref_agg)
    assert rows == [lv[0].shape[0] for lv in levels], (rows, [lv[0].shape[0] for lv in levels])
    ref_nnz = [lv[0].nnz for lv in levels]
    assert nnz[0] == ref_nnz[0]
    for a, b in zip(nnz, ref_nnz):
        assert abs(a - b) <= 1e-3 * b, (nnz, ref_nnz)
