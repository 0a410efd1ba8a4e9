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


def markov_steps(phi, P0, steps):
    """Discrete-time diffusion p_{k+1} = p_k P (Sec. "Simulating discrete-time
    diffusion"), for the distributions stored as the columns of P0 (column j = p_0^T):
    each step multiplies by P^T.  Returns the columns after `steps` steps."""
    P = markov_transition(phi)
    X = np.array(P0, dtype=np.float64)
    for _ in range(steps):
        X = P.T @ X
    return X


def markov_spectrum(phi):
    """Eigenvalues of P = diag(w)^{-1} phi in increasing order, from the symmetric
    matrix diag(w)^{-1/2} phi diag(w)^{-1/2} that is similar to P (w > 0)."""
    w = walk_degree(phi)
    r = 1.0 / np.sqrt(w)
    S = r[:, None] * phi * r[None, :]
    return np.linalg.eigvalsh(0.5 * (S + S.T))


def spectral_gap(phi):
    """(lambda_2, lambda_min, gap) of the chain: lambda_2 is the largest eigenvalue of P
    below the top one (1, eigenvector 1), lambda_min the smallest, and the gap separates
    1 from the next eigenvalue in modulus: gap = 1 - max(|lambda_2|, |lambda_min|)
    (the quantity compared across Laplacians in the tree experiment of Sec. 5)."""
    lam = markov_spectrum(phi)
    lam2, lmin = lam[-2], lam[0]
    return float(lam2), float(lmin), float(1.0 - max(abs(lam2), abs(lmin)))
