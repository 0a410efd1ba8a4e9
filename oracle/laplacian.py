"""Walk Laplacians, diffusion and Markov chains from a dense phi (float64).

Test infrastructure: see the package docstring.
"""

import numpy as np


def walk_degree(phi):
    """w = phi 1, the total communicability t(f) = f(A) 1 (Sec. 3.1) and its BTDW analogue."""
    return phi.sum(axis=1)


def walk_laplacian(phi):
    """L = diag(phi 1) - phi (eq. f-laplacian, eq. weighted_laplacian)."""
    return np.diag(walk_degree(phi)) - phi


def apply_laplacian(phi, X):
    """L X = w * X - phi X, the product the library computes without forming L."""
    w = walk_degree(phi)
    return w[:, None] * X - phi @ X


def expv(Lap, U0, ts):
    """exp(-t L) U0 for each t, from the eigendecomposition of the symmetric L
    (diffusion p(t) = p0 exp(-t L), eq. diffusion_on_G; L symmetric so the
    row-vector and column-vector forms are transposes of each other)."""
    lam, V = np.linalg.eigh(Lap)
    C = V.T @ U0
    return [V @ (np.exp(-t * lam)[:, None] * C) for t in np.atleast_1d(ts)]


def return_probabilities(Lap, t):
    """diag exp(-t L): return probabilities [P(t)]_jj (Sec. 4.4)."""
    lam, V = np.linalg.eigh(Lap)
    return (V * V) @ np.exp(-t * lam)


def average_return_probability(Lap, t):
    """p_hat(t) = tr exp(-t L) / n (eq. average_return_probabilities)."""
    return float(return_probabilities(Lap, t).mean())


def markov_transition(phi):
    """P = I - Dd^{-1} L (eq. let_there_be_markov).

    Reading: Dd = diag(w) with w = phi 1 ("a single evaluation of the matrix
    function"), so P = diag(w)^{-1} phi.  The literal diag(L) = w - diag(phi)
    does not reproduce the paper's Fig. 1; diag(w) does, to every printed digit.
    """
    w = walk_degree(phi)
    return phi / w[:, None]


def stationary_distribution(phi):
    """pi = w / sum(w): pi P = 1^T phi / sum(w) = pi since phi is symmetric."""
    w = walk_degree(phi)
    return w / w.sum()
