"""Pins of the oracle's local node features (oracle.features.features): hand-derived
counts on small graphs whose structure fixes them, and brute-force enumeration on
random graphs (triangles over node triples, clustering as the fraction of connected
neighbour pairs, neighbour-degree statistics by explicit loops).

Feature order: log1p(s d), log1p(s^2 d), log1p(s^3 2t), log1p(s^2 S2), log1p(s mean),
log1p(s rms), log1p(s max), clustering; d degree, t triangles through the node, S2 the
sum of neighbour degrees, mean / rms / max over the neighbours' degrees.
"""

import itertools
import math

import numpy as np
import pytest

import synth
from oracle import features as F
from oracle import walks


def expected(s, d, t, S2, mean, rms, mx, cc):
    d, t, S2, mean, rms, mx, cc = (np.asarray(v, dtype=float) for v in (d, t, S2, mean, rms, mx, cc))
    return np.stack([np.log1p(s * d), np.log1p(s * s * d), np.log1p(s ** 3 * 2 * t), np.log1p(s * s * S2),
                     np.log1p(s * mean), np.log1p(s * rms), np.log1p(s * mx), cc], axis=1)


def csr(n, edges):
    u = np.array([a for a, _ in edges])
    v = np.array([b for _, b in edges])
    return synth.graphs.csr_from_edges(n, u, v)


@pytest.mark.parametrize("s", [1.0, 0.3])
def test_g58_hand_values(s):
    """G_{5,8} of Fig. 1: path 1-2-3-4-5 with 8 leaves on node 3 (a tree: no triangles).
    Degrees 1, 2, 10, 2, 1 on the path and 1 on the leaves; neighbour degrees
    node 1: {2}; node 2: {1, 10}; node 3: {2, 2, 1 x 8}; node 4: {10, 1}; node 5: {2};
    leaf: {10}."""
    rp, ci = synth.toy_g58()
    got = F.features(13, rp, ci, s)
    leaf = (1, 0, 10, 10.0, 10.0, 10, 0.0)
    rows = [
        (1, 0, 2, 2.0, 2.0, 2, 0.0),
        (2, 0, 11, 5.5, math.sqrt(50.5), 10, 0.0),
        (10, 0, 12, 1.2, math.sqrt(1.6), 2, 0.0),
        (2, 0, 11, 5.5, math.sqrt(50.5), 10, 0.0),
        (1, 0, 2, 2.0, 2.0, 2, 0.0),
    ] + [leaf] * 8
    ref = expected(s, *zip(*rows))
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)


def test_complete_graph_k4():
    """K4: degree 3, three triangles through every node, every neighbour pair joined."""
    n = 4
    rp, ci = csr(n, list(itertools.combinations(range(n), 2)))
    got = F.features(n, rp, ci, 0.5)
    ref = expected(0.5, [3] * 4, [3] * 4, [9] * 4, [3] * 4, [3] * 4, [3] * 4, [1] * 4)
    np.testing.assert_allclose(got, ref, rtol=1e-14)


def test_diamond():
    """K4 minus the edge a-d: triangles abc and bcd; b and c see 2 of their 3 neighbour
    pairs joined (clustering 2/3), a and d their only pair (1)."""
    a, b, c, d = range(4)
    rp, ci = csr(4, [(a, b), (a, c), (b, c), (b, d), (c, d)])
    got = F.features(4, rp, ci, 1.0)
    ref = expected(1.0, [2, 3, 3, 2], [1, 2, 2, 1], [6, 7, 7, 6], [3, 7 / 3, 7 / 3, 3],
                   [3, math.sqrt(17 / 3), math.sqrt(17 / 3), 3], [3, 3, 3, 3], [1, 2 / 3, 2 / 3, 1])
    np.testing.assert_allclose(got, ref, rtol=1e-14)


@pytest.mark.parametrize("k", [2, 5, 9])
def test_star(k):
    """Star K_{1,k}: centre of degree k whose neighbours all have degree 1; leaves of
    degree 1 whose one neighbour has degree k; no triangles."""
    rp, ci = csr(k + 1, [(0, j) for j in range(1, k + 1)])
    got = F.features(k + 1, rp, ci, 1.0)
    ref = expected(1.0, [k] + [1] * k, [0] * (k + 1), [k] * (k + 1), [1.0] + [k] * k, [1.0] + [k] * k,
                   [1] + [k] * k, [0.0] * (k + 1))
    np.testing.assert_allclose(got, ref, rtol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 7])
def test_cycle(n):
    """Cycle C_n: degree 2 everywhere; the triangle C_3 has one triangle per node and
    clustering 1, longer cycles none."""
    rp, ci = csr(n, [(i, (i + 1) % n) for i in range(n)])
    got = F.features(n, rp, ci, 1.0)
    t = 1 if n == 3 else 0
    ref = expected(1.0, [2] * n, [t] * n, [4] * n, [2] * n, [2] * n, [2] * n, [float(t)] * n)
    np.testing.assert_allclose(got, ref, rtol=1e-14)


def test_isolated_nodes_are_zero():
    rp, ci = csr(5, [(0, 1)])
    got = F.features(5, rp, ci, 1.0)
    assert np.all(got[2:] == 0.0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_graphs_against_enumeration(seed):
    """Brute force on G(40, 160) and a power-law graph: triangles over node triples,
    clustering as connected neighbour pairs / all neighbour pairs, neighbour-degree
    statistics by loops over adjacency lists."""
    if seed == 3:
        n = 60
        rp, ci = synth.configuration_model_powerlaw(n, 2.5, 2, 12, 5)
    else:
        n = 40
        rp, ci = synth.erdos_renyi_gnm(n, 160, seed)
    A = walks.adjacency(n, rp, ci)
    nbrs = [list(np.nonzero(A[i])[0]) for i in range(n)]
    deg = np.array([len(v) for v in nbrs], dtype=float)
    tri = np.zeros(n)
    for i, j, k in itertools.combinations(range(n), 3):
        if A[i, j] and A[j, k] and A[i, k]:
            tri[[i, j, k]] += 1
    assert tri.sum() > 0
    S2 = np.array([sum(deg[j] for j in v) for v in nbrs])
    mean = np.array([np.mean([deg[j] for j in v]) if v else 0.0 for v in nbrs])
    rms = np.array([math.sqrt(np.mean([deg[j] ** 2 for j in v])) if v else 0.0 for v in nbrs])
    mx = np.array([max(deg[j] for j in v) if v else 0.0 for v in nbrs])
    cc = np.zeros(n)
    for i, v in enumerate(nbrs):
        pairs = list(itertools.combinations(v, 2))
        if pairs:
            cc[i] = sum(1 for a, b in pairs if A[a, b]) / len(pairs)
    s = 0.7
    np.testing.assert_allclose(F.features(n, rp, ci, s), expected(s, deg, tri, S2, mean, rms, mx, cc), rtol=1e-13)
