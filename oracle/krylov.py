"""Same-K block Krylov reference in float64 (test infrastructure).

The Krylov route of Sec. 4.1 written plainly: block Lanczos on a symmetric operator
from a start block X,

    X = V_0 R_0,    Op V_j = V_{j-1} B_{j-1}^T + V_j A_j + V_{j+1} B_j,

then f(Op) X ~ [V_0 .. V_{K-1}] f(T_K) E_1 R_0 with T_K the (K b) x (K b) block
tridiagonal matrix of the A_j (diagonal) and B_j (below the diagonal).  With the same
start block and the same K as the GPU path this is the same approximation computed in
exact-as-possible arithmetic, which separates the kernels' rounding (GPU against this
reference) from the method's truncation error (this reference against the exact
function).  Used for graphs beyond dense sizes.

Plain choices, written for checking by eye rather than speed:
  * each new block is orthogonalised by classical Gram-Schmidt run twice, against the
    two previous blocks ("local") or every earlier block ("full");
  * it is then orthonormalised through its thin SVD, W = U S Q^T, V = U, B = S Q^T,
    with directions below `defl` times the block's scale dropped (their basis column is
    zero).  This spans the same space as the CholQR2 factorisation the library uses;
    the Galerkin approximation V f(T) V^T X depends only on the space, not on the
    orthonormal basis chosen for it;
  * f(T) from the eigendecomposition of T (numpy eigh).

Sparse products go through scipy.sparse, split over row chunks on a thread pool
(`spmm`), which computes exactly the plain product.
"""

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_POOL = None


def threads():
    """Host threads used for the row-chunked sparse products: the CPUs the process may
    run on, capped by OMP_NUM_THREADS when that is set (the host's share of a shared
    machine)."""
    try:
        nt = max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        nt = max(1, os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS", "")
    if cap.isdigit() and int(cap) > 0:
        nt = min(nt, int(cap))
    return nt


def spmm(A, X):
    """A @ X for a scipy CSR A and a dense block X, rows split over a thread pool."""
    global _POOL
    n = A.shape[0]
    nt = threads()
    if nt == 1 or n < 4096:
        return A @ X
    if _POOL is None:
        _POOL = ThreadPoolExecutor(nt)
    cuts = np.linspace(0, n, 4 * nt + 1).astype(np.int64)
    parts = list(_POOL.map(lambda k: A[cuts[k]:cuts[k + 1]] @ X, range(4 * nt)))
    return np.vstack(parts)


def orthonormalise(W, scale, defl):
    """W = V B with V^T V = diag(kept) (dropped directions give zero columns) and B b x b."""
    U, s, Qt = np.linalg.svd(W, full_matrices=False)
    keep = s > defl * scale
    V = U * keep
    B = (s * keep)[:, None] * Qt
    return V, B


def block_lanczos(apply_op, X, K, reorth="local", defl=1e-12):
    """K block Lanczos steps on the symmetric operator apply_op from X (n x b).

    Returns (V, A, B, R0): V the K + 1 blocks, A_j = V_j^T Op V_j (symmetrised), B_j
    the coupling V_{j+1} B_j of step j (B_{K-1} is the residual coupling), X = V_0 R0.
    """
    X = np.asarray(X, dtype=np.float64)
    n, b = X.shape
    scale0 = np.linalg.norm(X, 2)
    basis = np.zeros((n, (K + 1) * b))  # V_j is columns [j b, (j + 1) b)
    V = [basis[:, j * b:(j + 1) * b] for j in range(K + 1)]
    V[0][:], R0 = orthonormalise(X, scale0, defl)
    A, B = [], []
    for j in range(K):
        W = apply_op(V[j])
        if j > 0:
            W = W - V[j - 1] @ B[j - 1].T
        Aj = V[j].T @ W
        Aj = 0.5 * (Aj + Aj.T)
        W = W - V[j] @ Aj
        scale = max(np.linalg.norm(W, 2), 1e-300)
        lo = 0 if reorth == "full" else max(0, j - 1)
        prev = basis[:, lo * b:(j + 1) * b]  # the blocks W is made orthogonal to
        for _ in range(2):  # classical Gram-Schmidt, twice
            W = W - prev @ (prev.T @ W)
        V[j + 1][:], Bj = orthonormalise(W, max(scale, np.linalg.norm(Aj, 2)), defl)
        A.append(Aj)
        B.append(Bj)
    return V, A, B, R0


def block_tridiagonal(A, B):
    """T with diagonal blocks A_j and T_{j+1, j} = B_j, T_{j, j+1} = B_j^T (K blocks)."""
    K, b = len(A), A[0].shape[0]
    T = np.zeros((K * b, K * b))
    for j in range(K):
        T[j * b:(j + 1) * b, j * b:(j + 1) * b] = A[j]
        if j + 1 < K:
            T[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = B[j]
            T[j * b:(j + 1) * b, (j + 1) * b:(j + 2) * b] = B[j].T
    return T


def projected_function(V, A, B, R0, K, f):
    """F = f(T_K) E_1 R_0 on the basis columns that were kept (a dropped direction has a
    zero basis column and a zero row and column of T; it is left out of T so that f is
    never evaluated on that artificial zero eigenvalue).  Returns (F, lam, U, kept)."""
    b = R0.shape[0]
    kept = np.concatenate([np.any(V[j] != 0.0, axis=0) for j in range(K)])
    T = block_tridiagonal(A, B)[np.ix_(kept, kept)]
    E1R0 = np.zeros((K * b, R0.shape[1]))
    E1R0[:b] = R0
    lam, U = np.linalg.eigh(T)
    F = np.zeros((K * b, R0.shape[1]))
    F[kept] = U @ (f(lam)[:, None] * (U.T @ E1R0[kept]))
    return F, lam, U, kept


def lanczos_function(apply_op, X, K, f, reorth="local", defl=1e-12):
    """f(Op) X ~ V_K f(T_K) E_1 R_0 after K block Lanczos steps (Sec. 4.1).  f acts on an
    array of eigenvalues.  Returns (Y, lanczos data)."""
    V, A, B, R0 = block_lanczos(apply_op, X, K, reorth, defl)
    b = X.shape[1]
    F, _, _, _ = projected_function(V, A, B, R0, K, f)
    Y = sum(V[j] @ F[j * b:(j + 1) * b] for j in range(K))
    return Y, (V, A, B, R0)


def deformed_apply(A, mu, alpha):
    """V -> A_mu(alpha) V = (1 - mu^2 alpha^2) V - alpha A V + alpha^2 mu D V (eq. deformed)."""
    d = np.asarray(A.sum(axis=1)).ravel()[:, None]
    c0 = 1.0 - mu * mu * alpha * alpha
    return lambda V: c0 * V - alpha * spmm(A, V) + alpha * alpha * mu * d * V


def phi_resolvent_lanczos(A, mu, alpha, X, K, reorth="local"):
    """phi X = (1 - mu^2 alpha^2) A_mu(alpha)^{-1} X by K block Lanczos steps on the
    deformed Laplacian (the library's Lanczos resolvent)."""
    s = 1.0 - mu * mu * alpha * alpha
    Y, _ = lanczos_function(deformed_apply(A, mu, alpha), X, K, lambda x: s / x, reorth)
    return Y


def phi_exp_lanczos(A, beta, X, K, reorth="local"):
    """phi X = exp(beta A) X at mu = 0 by K block Lanczos steps on A."""
    Y, _ = lanczos_function(lambda V: spmm(A, V), X, K, lambda x: np.exp(beta * x), reorth)
    return Y


def series_apply(A, mu, coeffs, X):
    """sum_k coeffs[k] q_k(A) X by eq. qrec on the block: q_2 X = A (A X) - mu D X, then
    q_{k+1} X = A q_k X + mu (mu I - D) q_{k-1} X."""
    d = np.asarray(A.sum(axis=1)).ravel()[:, None]
    X = np.asarray(X, dtype=np.float64)
    out = coeffs[0] * X
    if len(coeffs) == 1:
        return out
    q_prev, q_cur = X, spmm(A, X)
    out = out + coeffs[1] * q_cur
    for k in range(1, len(coeffs) - 1):
        q_next = spmm(A, q_cur) - mu * d * q_prev if k == 1 else spmm(A, q_cur) + mu * (mu - d) * q_prev
        out = out + coeffs[k + 1] * q_next
        q_prev, q_cur = q_cur, q_next
    return out


def exp_coefficients(beta, K):
    return np.array([beta ** k / math.factorial(k) for k in range(K + 1)])


def expv_lanczos(apply_phi, w, U0, ts, K, reorth="full"):
    """exp(-t L) U0 for every t from one outer block Lanczos basis on the walk Laplacian
    L V = w * V - phi V (eq. f-laplacian; eq. diffusion_on_G_with_downweighted_walk),
    with phi V by apply_phi (the inner evaluation).  Returns (list of Y(t), list of the
    a-posteriori estimates ||B_{K-1} F_{K-1}(t)||_F, F(t) = exp(-t T) E_1 R_0)."""
    w = np.asarray(w, dtype=np.float64)[:, None]
    V, A, B, R0 = block_lanczos(lambda X: w * X - apply_phi(X), U0, K, reorth)
    b = U0.shape[1]
    Ys, errs = [], []
    for t in ts:
        F, _, _, _ = projected_function(V, A, B, R0, K, lambda x: np.exp(-t * x))
        Ys.append(sum(V[j] @ F[j * b:(j + 1) * b] for j in range(K)))
        errs.append(float(np.linalg.norm(B[K - 1] @ F[(K - 1) * b:K * b])))
    return Ys, errs
