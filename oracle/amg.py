"""Aggregation AMG-preconditioned conjugate gradients on the deformed Laplacian
(test infrastructure).

Sec. 4.2 solves the resolvent systems A_mu(alpha) y = x (eq. deformed; an M-matrix for
alpha rho(Z_mu) < 1) by CG preconditioned with an aggregation multigrid: Vanek-Mandel-
Brezina aggregation, a V-cycle with one sweep of l1-Jacobi before and after the coarse
correction, and 30 sweeps of the smoother as the coarsest-level solver; Sec. 5.3 runs
CG to a relative tolerance of 1e-9.  Written here from those descriptions with scipy
sparse matrices, one level at a time:

  * strength: j is strongly coupled to i (j != i) when |a_ij| >= theta sqrt(a_ii a_jj);
  * aggregation (Vanek, Mandel, Brezina 1996), over the nodes that have at least one
    strong neighbour (the others are left to the smoother and get no coarse unknown):
      1. in node order, a node whose strong neighbourhood (itself and its strong
         neighbours) holds no aggregated node becomes the root of a new aggregate made
         of that neighbourhood;
      2. every node still free joins the aggregate (as formed in step 1) of its most
         strongly coupled neighbour among those step 1 aggregated (largest |a_ij|,
         ties to the lower index);
      3. in node order, every node still free forms a new aggregate with its free strong
         neighbours;
  * tentative prolongator: piecewise constant on the aggregates, columns scaled to unit
    norm (the constant vector is the near-kernel the aggregates reproduce);
  * smoothed prolongator P = (I - omega D^-1 A) P_tent with omega = 4 / (3 ||D^-1 A||_inf)
    (the infinity norm bounds the spectral radius of D^-1 A);
  * Galerkin coarse matrix A_c = P^T A P; levels are added while the coarse size shrinks
    below 0.9 of the fine one and stays above `coarse_size`;
  * l1-Jacobi: x <- x + M^-1 (b - A x), M = diag(sum_j |a_ij|) (the l1 smoother with
    every row its own block; M^-1 A has its spectrum in (0, 1] for these matrices, so the
    sweeps converge and the V-cycle is symmetric positive definite).
"""

import numpy as np
import scipy.sparse as sp


def strength(A, theta):
    """Boolean CSR pattern of the strong couplings (diagonal excluded)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    C = A.tocoo()
    off = C.row != C.col
    r, c, v = C.row[off], C.col[off], C.data[off]
    keep = np.abs(v) >= theta * np.sqrt(np.abs(d[r] * d[c]))
    S = sp.csr_matrix((np.ones(int(keep.sum())), (r[keep], c[keep])), shape=A.shape)
    S.sort_indices()
    return S


def vmb_aggregate(A, theta):
    """Aggregate index of every node (-1: no strong neighbour, left out) and the number
    of aggregates."""
    A = sp.csr_matrix(A)
    S = strength(A, theta)
    n = A.shape[0]
    agg = -np.ones(n, dtype=np.int64)
    nbrs = [S.indices[S.indptr[i]:S.indptr[i + 1]] for i in range(n)]
    active = np.array([nb.size > 0 for nb in nbrs])
    k = 0
    for i in range(n):  # 1: roots with wholly free neighbourhoods
        if active[i] and agg[i] < 0 and np.all(agg[nbrs[i]] < 0):
            agg[i] = k
            agg[nbrs[i]] = k
            k += 1
    first = agg.copy()
    Ad = A.tolil()
    for i in range(n):  # 2: join the most strongly coupled aggregate of step 1
        if active[i] and agg[i] < 0:
            best, bestv = -1, -1.0
            for j in nbrs[i]:
                if first[j] >= 0 and abs(Ad[i, j]) > bestv:
                    best, bestv = j, abs(Ad[i, j])
            if best >= 0:
                agg[i] = first[best]
    for i in range(n):  # 3: leftovers with their free strong neighbours
        if active[i] and agg[i] < 0:
            free = [j for j in nbrs[i] if agg[j] < 0]
            agg[i] = k
            agg[free] = k
            k += 1
    return agg, k


def tentative_prolongator(agg, nagg):
    n = agg.size
    rows = np.nonzero(agg >= 0)[0]
    sizes = np.bincount(agg[rows], minlength=nagg).astype(np.float64)
    vals = 1.0 / np.sqrt(sizes[agg[rows]])
    return sp.csr_matrix((vals, (rows, agg[rows])), shape=(n, nagg))


def smoothed_prolongator(A, Pt):
    A = sp.csr_matrix(A)
    d = A.diagonal()
    Dinv_A = sp.diags(1.0 / d) @ A
    omega = 4.0 / (3.0 * np.abs(Dinv_A).sum(axis=1).max())
    return sp.csr_matrix(Pt - omega * (Dinv_A @ Pt)), omega


def l1_diagonal(A):
    return np.asarray(np.abs(sp.csr_matrix(A)).sum(axis=1)).ravel()


def hierarchy(A, theta=0.01, coarse_size=256, max_levels=20):
    """Levels [(A_l, P_l, m_l)] with P_l the prolongator from level l + 1 (None on the
    last level) and m_l the l1 diagonal."""
    levels = []
    A = sp.csr_matrix(A)
    while True:
        m = l1_diagonal(A)
        n = A.shape[0]
        if n <= coarse_size or len(levels) + 1 >= max_levels:
            levels.append((A, None, m))
            break
        agg, nagg = vmb_aggregate(A, theta)
        if nagg == 0 or nagg > 0.9 * n:
            levels.append((A, None, m))
            break
        P, _ = smoothed_prolongator(A, tentative_prolongator(agg, nagg))
        levels.append((A, P, m))
        A = sp.csr_matrix(P.T @ A @ P)
    return levels


def vcycle(levels, b, l=0, coarse_sweeps=30):
    """One V-cycle from a zero initial guess at level l: one l1-Jacobi sweep, coarse
    correction of the residual, one sweep; the coarsest level takes coarse_sweeps
    sweeps."""
    A, P, m = levels[l]
    m = m[:, None] if b.ndim == 2 else m
    if P is None:
        x = np.zeros_like(b)
        for _ in range(coarse_sweeps):
            x = x + (b - A @ x) / m
        return x
    x = b / m
    r = b - A @ x
    x = x + P @ vcycle(levels, P.T @ r, l + 1, coarse_sweeps)
    return x + (b - A @ x) / m


def pcg(A, B, levels, tol=1e-9, maxiter=1000):
    """Column-wise preconditioned CG from x = 0, stopping each column when its residual
    norm drops below tol times the norm of its right-hand side.  Returns (X, the
    iteration count of every column)."""
    A = sp.csr_matrix(A)
    B = np.asarray(B, dtype=np.float64)
    B2 = B if B.ndim == 2 else B[:, None]
    X = np.zeros_like(B2)
    its = np.zeros(B2.shape[1], dtype=np.int64)
    for c in range(B2.shape[1]):
        b = B2[:, c]
        x = np.zeros_like(b)
        r = b.copy()
        nb = np.linalg.norm(b)
        if nb == 0.0:
            continue
        z = vcycle(levels, r)
        p = z.copy()
        rz = r @ z
        for k in range(1, maxiter + 1):
            q = A @ p
            a = rz / (p @ q)
            x = x + a * p
            r = r - a * q
            its[c] = k
            if np.linalg.norm(r) <= tol * nb:
                break
            z = vcycle(levels, r)
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
        X[:, c] = x
    return (X if B.ndim == 2 else X[:, 0]), its
