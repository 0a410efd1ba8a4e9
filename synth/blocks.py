"""Seeded dense blocks (row-major n x b) used as right-hand sides and probes."""

import numpy as np


def gaussian_block(n, b, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal((n, b)).astype(dtype))


def rademacher_block(n, b, seed, dtype=np.float64):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, 2, size=(n, b), dtype=np.int8)
    return np.ascontiguousarray((2.0 * s - 1.0).astype(dtype))


def spike_block(n, nodes, dtype=np.float64):
    """Column j is the unit vector at ``nodes[j]``."""
    nodes = np.atleast_1d(np.asarray(nodes, dtype=np.int64))
    X = np.zeros((n, nodes.size), dtype=dtype)
    X[nodes, np.arange(nodes.size)] = 1.0
    return X


def sparse_initial_block(n, b, nnz_per_col, seed, candidates=None, dtype=np.float64):
    """b probability vectors, each with mass 1/nnz_per_col on nnz_per_col random nodes.

    ``candidates`` restricts the support (e.g. to non-isolated nodes)."""
    rng = np.random.default_rng(seed)
    pool = np.arange(n) if candidates is None else np.asarray(candidates)
    X = np.zeros((n, b), dtype=dtype)
    for j in range(b):
        sel = rng.choice(pool.size, size=nnz_per_col, replace=False)
        X[pool[sel], j] = 1.0 / nnz_per_col
    return X


def glorot_params(shapes, seed):
    """Seeded Glorot-uniform weights for every 2-D shape, zeros for 1-D shapes,
    concatenated in order (initial weights for the control-variate network)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes:
        if len(s) == 2:
            lim = np.sqrt(6.0 / (s[0] + s[1]))
            parts.append(rng.uniform(-lim, lim, size=s).ravel())
        else:
            parts.append(np.zeros(int(np.prod(s))))
    return np.concatenate(parts)
