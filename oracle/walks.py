"""Walk-count matrices, dense float64 (paper Sec. 2 and Sec. 3.2).

Test infrastructure: see the package docstring.
"""

import numpy as np


def adjacency(n, rowptr, colidx):
    """Dense 0/1 adjacency matrix of a simple graph (Definition "adjacency", Sec. 2)."""
    A = np.zeros((n, n), dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(np.asarray(rowptr)))
    A[rows, np.asarray(colidx, dtype=np.int64)] = 1.0
    return A


def degrees(A):
    """d = A 1, the diagonal of the degree matrix D (Definition of L = D - A, Sec. 2.1)."""
    return A.sum(axis=1)


def btdw_counts(A, mu, kmax):
    """Backtrack-downweighted walk-count matrices q_0 .. q_kmax (Sec. 3.2, eq. qrec).

    q_0 = I, q_1 = A, q_2 = A^2 - mu D, and q_{k+1} = A q_k + mu (mu I - D) q_{k-1}.

    Reading: the three-term recurrence produces q_3 onward (k >= 2).  q_2 is a
    separate initial term; applying the recurrence at k = 1 would add mu^2 I,
    which the weighted-walk definition (each backtrack i_l = i_{l+2} weighted
    by 1 - mu) does not contain.  This matches the nonbacktracking special case
    eq. Br, which is stated for k >= 3.
    """
    n = A.shape[0]
    D = np.diag(degrees(A))
    I = np.eye(n)
    q = [I, A.copy()]
    if kmax >= 2:
        q.append(A @ A - mu * D)
    for k in range(2, kmax):
        q.append(A @ q[k] + mu * (mu * I - D) @ q[k - 1])
    return q[: kmax + 1]


def nbt_counts(A, kmax):
    """Nonbacktracking walk counts p_0 .. p_kmax (Sec. 3.2, eq. Br):
    p_0 = I, p_1 = A, p_2 = A^2 - D, p_k = A p_{k-1} + (I - D) p_{k-2} for k >= 3."""
    n = A.shape[0]
    D = np.diag(degrees(A))
    I = np.eye(n)
    p = [I, A.copy()]
    if kmax >= 2:
        p.append(A @ A - D)
    for k in range(3, kmax + 1):
        p.append(A @ p[k - 1] + (I - D) @ p[k - 2])
    return p[: kmax + 1]


def linearisation(A, mu):
    """The 2n x 2n matrix Z = [[O, I], [mu (mu I - D), A]] of Proposition
    "whe-we-converge" (eq. Zdef)."""
    n = A.shape[0]
    D = np.diag(degrees(A))
    Z = np.zeros((2 * n, 2 * n))
    Z[:n, n:] = np.eye(n)
    Z[n:, :n] = mu * (mu * np.eye(n) - D)
    Z[n:, n:] = A
    return Z


def spectral_radius(M):
    """rho(M) by a dense eigenvalue computation."""
    return float(np.max(np.abs(np.linalg.eigvals(M))))
