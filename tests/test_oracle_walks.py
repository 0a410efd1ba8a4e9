"""Pins of the oracle's walk counts (Sec. 3.2) against brute-force enumeration,
the mu = 0 and mu = 1 limits, and the Z identity of Prop. "whe-we-converge"."""

import itertools

import numpy as np
import pytest

import synth
from oracle import walks


def small_graphs():
    # 7 nodes: a triangle 0-1-2, a 4-cycle 2-3-4-5, a pendant 6 on node 0
    tri = synth.csr_from_edges(7, [0, 1, 2, 2, 3, 4, 5, 0], [1, 2, 0, 3, 4, 5, 2, 6])
    return {
        "irregular7": (7,) + tri,
        "star4": (5,) + synth.star_graph(4),
        "cycle5": (5,) + synth.cycle_graph(5),
        "path4": (4,) + synth.csr_from_edges(4, [0, 1, 2], [1, 2, 3]),
        "k4": (4,) + synth.complete_graph(4),
    }


def brute_force_weighted_walks(A, k, mu):
    """Sum over all walks i_0..i_k of (1 - mu)^(number of l with i_l = i_{l+2}),
    the weighted count that defines q_k (Sec. 3.2)."""
    n = A.shape[0]
    adj = [np.nonzero(A[i])[0] for i in range(n)]
    Q = np.zeros((n, n))
    theta = 1.0 - mu

    def rec(walk):
        if len(walk) == k + 1:
            bt = sum(1 for l in range(len(walk) - 2) if walk[l] == walk[l + 2])
            Q[walk[0], walk[-1]] += theta ** bt
            return
        for j in adj[walk[-1]]:
            rec(walk + [j])

    for i in range(n):
        rec([i])
    return Q


@pytest.mark.parametrize("name", list(small_graphs()))
@pytest.mark.parametrize("mu", [0.0, 0.3, 1.0])
def test_btdw_counts_match_enumeration(name, mu):
    n, rp, ci = small_graphs()[name]
    A = walks.adjacency(n, rp, ci)
    q = walks.btdw_counts(A, mu, 6)
    for k in range(7):
        if k == 0:
            ref = np.eye(n)
        else:
            ref = brute_force_weighted_walks(A, k, mu)
        np.testing.assert_allclose(q[k], ref, rtol=0, atol=1e-12, err_msg=f"k={k}")


@pytest.mark.parametrize("name", list(small_graphs()))
def test_nbt_counts_are_integer_nonbacktracking_walks(name):
    n, rp, ci = small_graphs()[name]
    A = walks.adjacency(n, rp, ci)
    p = walks.nbt_counts(A, 6)
    for k in range(1, 7):
        np.testing.assert_array_equal(p[k], brute_force_weighted_walks(A, k, 1.0))


@pytest.mark.parametrize("name", list(small_graphs()))
def test_mu_limits(name):
    n, rp, ci = small_graphs()[name]
    A = walks.adjacency(n, rp, ci)
    q0 = walks.btdw_counts(A, 0.0, 7)
    for k in range(8):
        np.testing.assert_array_equal(q0[k], np.linalg.matrix_power(A, k))
    q1 = walks.btdw_counts(A, 1.0, 7)
    p = walks.nbt_counts(A, 7)
    for k in range(8):
        np.testing.assert_array_equal(q1[k], p[k])


def test_recurrence_start_reading():
    """Applying eq. qrec already at k = 1 would give A^2 + mu^2 I - mu D for q_2,
    which disagrees with enumeration; the oracle's q_2 = A^2 - mu D agrees."""
    n, rp, ci = small_graphs()["irregular7"]
    A = walks.adjacency(n, rp, ci)
    mu = 0.3
    wrong = A @ A + mu * (mu * np.eye(n) - np.diag(A.sum(1)))
    ref = brute_force_weighted_walks(A, 2, mu)
    assert np.abs(wrong - ref).max() > 0.05
    np.testing.assert_allclose(walks.btdw_counts(A, mu, 2)[2], ref, atol=1e-14)


@pytest.mark.parametrize("mu", [0.0, 0.25, 0.75, 1.0])
def test_z_identity(mu):
    """Z^k [q_1; q_2] = [q_{k+1}; q_{k+2}] (proof of Prop. "whe-we-converge")."""
    n, rp, ci = small_graphs()["irregular7"]
    A = walks.adjacency(n, rp, ci)
    q = walks.btdw_counts(A, mu, 10)
    Z = walks.linearisation(A, mu)
    B = np.vstack([q[1], q[2]])
    for k in range(8):
        np.testing.assert_allclose(np.linalg.matrix_power(Z, k) @ B, np.vstack([q[k + 1], q[k + 2]]), atol=1e-9)


def test_walk_counts_symmetric_nonnegative():
    n, rp, ci = small_graphs()["irregular7"]
    A = walks.adjacency(n, rp, ci)
    for mu in (0.0, 0.5, 1.0):
        for qk in walks.btdw_counts(A, mu, 8):
            np.testing.assert_array_equal(qk, qk.T)
            assert qk.min() >= -1e-12
