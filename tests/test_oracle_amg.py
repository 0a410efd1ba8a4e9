"""Pins of the oracle's aggregation AMG and preconditioned CG (oracle.amg): hand-traced
aggregations, the algebra of the prolongators and Galerkin products, the smoother's
convergence, symmetry and definiteness of the V-cycle, and the PCG solution against a
direct solve."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import amg, sparse, walks


def deformed(n, rp, ci, mu, alpha):
    return sp.csr_matrix(sparse.deformed(sparse.adjacency(n, rp, ci), mu, alpha))


def path(n):
    return synth.csr_from_edges(n, np.arange(n - 1), np.arange(1, n))


def test_path_aggregation_by_hand():
    """P_7, every coupling strong: roots 0, 3, 6 take {0, 1}, {2, 3, 4}, {5, 6} (node 2's
    and 5's neighbourhoods already hold an aggregated node when their turn comes)."""
    rp, ci = path(7)
    A = deformed(7, rp, ci, 0.0, 0.3)
    agg, k = amg.vmb_aggregate(A, 0.01)
    assert k == 3 and agg.tolist() == [0, 0, 1, 1, 1, 2, 2]


def test_star_aggregation_by_hand():
    """Star with the centre numbered last: node 0 takes {0, centre}; the other leaves
    find the centre aggregated and join its aggregate in step 2 (one aggregate).  With
    the centre first it takes everything in step 1."""
    k = 5
    rp, ci = synth.csr_from_edges(k + 1, np.arange(k), np.full(k, k))
    agg, na = amg.vmb_aggregate(deformed(k + 1, rp, ci, 0.0, 0.2), 0.01)
    assert na == 1 and np.all(agg == 0)
    rp, ci = synth.csr_from_edges(k + 1, np.zeros(k, dtype=int), np.arange(1, k + 1))
    agg, na = amg.vmb_aggregate(deformed(k + 1, rp, ci, 0.0, 0.2), 0.01)
    assert na == 1 and np.all(agg == 0)


def test_relabelled_path_by_hand():
    """P_5 visited in the order of its labels 0, 2, 4, 1, 3 along the path 0-2-4-1-3:
    node 0 roots {0, 2}; node 1 (neighbours 4 and 3, all free) roots {1, 3, 4}.  (After
    step 1 every free node has a neighbour aggregated in step 1, the one that kept it
    from being a root, so step 2 places it and step 3 finds nothing here.)"""
    order = [0, 2, 4, 1, 3]
    rp, ci = synth.csr_from_edges(5, order[:-1], order[1:])
    agg, k = amg.vmb_aggregate(deformed(5, rp, ci, 0.0, 0.3), 0.01)
    assert agg.tolist() == [0, 1, 0, 1, 1] and k == 2


def test_weak_couplings_leave_nodes_out():
    rp, ci = path(6)
    A = deformed(6, rp, ci, 0.0, 0.001)  # |a_ij| = 1e-3 < 0.01 sqrt(a_ii a_jj)
    agg, k = amg.vmb_aggregate(A, 0.01)
    assert k == 0 and np.all(agg == -1)


@pytest.mark.parametrize("graph", ["ba", "grid"])
def test_aggregation_partition_properties(graph):
    if graph == "ba":
        rp, ci = synth.barabasi_albert(600, 3, 4)
        n = 600
    else:
        rp, ci = synth.road_grid(25, 25, 0.8, seed=3)
        n = len(rp) - 1
    A = deformed(n, rp, ci, 0.5, 0.3 / walks.spectral_radius(walks.linearisation(walks.adjacency(n, rp, ci), 0.5)))
    S = amg.strength(A, 0.01)
    agg, k = amg.vmb_aggregate(A, 0.01)
    active = np.diff(S.indptr) > 0
    assert np.all(agg[active] >= 0) and np.all(agg[~active] == -1)
    assert set(agg[active].tolist()) == set(range(k))
    # every aggregate is connected in the strength graph
    for a in range(k):
        nodes = np.nonzero(agg == a)[0]
        sub = S[nodes][:, nodes]
        ncomp, _ = sp.csgraph.connected_components(sub, directed=False)
        assert ncomp == 1, a


def test_prolongators_and_galerkin_product():
    rp, ci = synth.road_grid(12, 12, 0.9, seed=5)
    n = len(rp) - 1
    A = deformed(n, rp, ci, 1.0, 0.2)
    agg, k = amg.vmb_aggregate(A, 0.01)
    Pt = amg.tentative_prolongator(agg, k)
    np.testing.assert_allclose((Pt.T @ Pt).toarray(), np.eye(k), atol=1e-15)
    P, omega = amg.smoothed_prolongator(A, Pt)
    Ad = A.toarray()
    D = np.diag(Ad)
    omega_ref = 4.0 / (3.0 * np.max(np.abs(Ad).sum(1) / D))
    assert abs(omega - omega_ref) < 1e-15
    np.testing.assert_allclose(P.toarray(), Pt.toarray() - omega_ref * (Ad / D[:, None]) @ Pt.toarray(), atol=1e-14)
    levels = amg.hierarchy(A, coarse_size=10)
    assert len(levels) >= 2
    Ac = levels[1][0].toarray()
    Pd = levels[0][1].toarray()
    np.testing.assert_allclose(Ac, Pd.T @ Ad @ Pd, atol=1e-13)
    assert np.linalg.eigvalsh(Ac).min() > 0


def test_l1_smoother_converges():
    rp, ci = synth.barabasi_albert(300, 4, 8)
    A = deformed(300, rp, ci, 0.5, 0.9 / walks.spectral_radius(walks.linearisation(walks.adjacency(300, rp, ci), 0.5)))
    Ad = A.toarray()
    m = amg.l1_diagonal(A)
    ev = np.linalg.eigvals(Ad / m[:, None]).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12


@pytest.mark.parametrize("graph", ["ba", "grid"])
def test_vcycle_is_symmetric_positive_definite(graph):
    if graph == "ba":
        rp, ci = synth.barabasi_albert(250, 3, 6)
    else:
        rp, ci = synth.road_grid(16, 16, 0.85, seed=6)
    n = len(rp) - 1
    Adj = walks.adjacency(n, rp, ci)
    alpha = 0.95 / walks.spectral_radius(walks.linearisation(Adj, 1.0))
    A = deformed(n, rp, ci, 1.0, alpha)
    levels = amg.hierarchy(A, coarse_size=20)
    assert len(levels) >= 2
    B = amg.vcycle(levels, np.eye(n))
    np.testing.assert_allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_pcg_matches_direct_solve_and_beats_plain_cg():
    rp, ci = synth.road_grid(40, 40, 0.8, seed=9)
    n = len(rp) - 1
    Adj = walks.adjacency(n, rp, ci)
    mu = 1.0
    alpha = 0.99 / walks.spectral_radius(walks.linearisation(Adj, mu))
    A = deformed(n, rp, ci, mu, alpha)
    X = synth.gaussian_block(n, 3, 10)
    levels = amg.hierarchy(A, coarse_size=64)
    Y, its = amg.pcg(A, X, levels, tol=1e-9)
    ref = spla.splu(A.tocsc()).solve(X)
    assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-7
    for c in range(3):
        assert np.linalg.norm(X[:, c] - A @ Y[:, c]) <= 1e-9 * np.linalg.norm(X[:, c])
    plain = []
    for c in range(3):
        cnt = [0]
        spla.cg(A, X[:, c], rtol=1e-9, atol=0.0, maxiter=5000, callback=lambda _: cnt.__setitem__(0, cnt[0] + 1))
        plain.append(cnt[0])
    assert max(its) < min(plain), (its, plain)
    # levels shrink by at least 10 % each
    sizes = [lv[0].shape[0] for lv in levels]
    assert all(b <= 0.9 * a for a, b in zip(sizes, sizes[1:]))
