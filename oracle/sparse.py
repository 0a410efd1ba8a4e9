"""Sparse float64 routes for graphs too large for dense matrices.

These evaluate the same definitions as ``genfun``/``laplacian``, applied to a
block X, using scipy.sparse as the matrix-product primitive:
  * exponential weights: the truncated series sum_{k<=K} c_k q_k(A) X built
    with eq. qrec on the block (q_{k+1} X = A (q_k X) + mu (mu I - D)(q_{k-1} X)),
    with K chosen so that the tail bound of ``genfun.exp_tail_bound`` is below
    ``tol``;
  * resolvent weights: (1 - mu^2 alpha^2) A_mu(alpha)^{-1} X (eq. deformed,
    general mu) by a sparse direct solve (SuperLU), or conjugate gradients to a
    tight tolerance when the factorisation would be too large.
Spectral quantities use ARPACK (scipy.sparse.linalg.eigsh / eigs).
Test infrastructure: see the package docstring.
"""

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .genfun import exp_tail_bound


def adjacency(n, rowptr, colidx):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    data = np.ones(colidx.size, dtype=np.float64)
    return sp.csr_matrix((data, colidx, rowptr), shape=(n, n))


def degrees(A):
    return np.asarray(A.sum(axis=1)).ravel()


def lambda_max(A, tol=1e-13):
    """Largest eigenvalue of the symmetric adjacency matrix (= rho(A) for A >= 0)."""
    if A.shape[0] <= 2000:
        return float(np.linalg.eigvalsh(A.toarray())[-1])
    v0 = np.ones(A.shape[0])
    val = spla.eigsh(A, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False)
    return float(val[0])


def linearisation(A, mu):
    """Sparse Z = [[O, I], [mu (mu I - D), A]] (eq. Zdef)."""
    n = A.shape[0]
    d = degrees(A)
    I = sp.identity(n, format="csr")
    return sp.bmat([[None, I], [sp.diags(mu * (mu - d)), A]], format="csr")


def rho_Z(A, mu, tol=1e-12):
    """Spectral radius of Z (Prop. "whe-we-converge").  The Perron root of Z is
    real and dominant; ARPACK's largest-real-part eigenvalue is returned."""
    n = A.shape[0]
    if n <= 600:
        Z = linearisation(A, mu).toarray()
        return float(np.max(np.abs(np.linalg.eigvals(Z))))
    Z = linearisation(A, mu)
    vals = spla.eigs(Z, k=3, which="LR", tol=tol, return_eigenvectors=False, v0=np.ones(2 * n))
    return float(np.max(np.abs(vals)))


def series_apply(A, mu, coeffs, X):
    """sum_k coeffs[k] q_k(A) X by eq. qrec on the block (q_2 X = A (A X) - mu D X)."""
    d = degrees(A)[:, None]
    X = np.asarray(X, dtype=np.float64)
    out = coeffs[0] * X
    if len(coeffs) == 1:
        return out
    q_prev = X
    q_cur = A @ X
    out = out + coeffs[1] * q_cur
    for k in range(1, len(coeffs) - 1):
        if k == 1:
            q_next = A @ q_cur - mu * d * q_prev
        else:
            q_next = A @ q_cur + mu * (mu - d) * q_prev
        out = out + coeffs[k + 1] * q_next
        q_prev, q_cur = q_cur, q_next
    return out


def exp_degree_for(beta, lam, tol):
    K = 1
    while exp_tail_bound(beta, lam, K) > tol:
        K += 1
    return K


def phi_exp_apply(A, mu, beta, X, tol=1e-17, K=None):
    """phi X for c_k = beta^k / k!, truncated where the tail bound drops below tol."""
    if K is None:
        K = exp_degree_for(beta, lambda_max(A), tol)
    coeffs = np.array([beta ** k / math.factorial(k) for k in range(K + 1)])
    return series_apply(A, mu, coeffs, X)


def deformed(A, mu, alpha):
    n = A.shape[0]
    d = degrees(A)
    return sp.diags((1.0 - mu * mu * alpha * alpha) + alpha * alpha * mu * d) - alpha * A


def phi_res_apply(A, mu, alpha, X, rtol=1e-14, direct_max_n=3000):
    """(1 - mu^2 alpha^2) A_mu(alpha)^{-1} X (eq. deformed, general mu)."""
    M = deformed(A, mu, alpha).tocsc()
    X = np.asarray(X, dtype=np.float64)
    s = 1.0 - mu * mu * alpha * alpha
    if A.shape[0] <= direct_max_n:
        lu = spla.splu(M)
        return s * lu.solve(X)
    out = np.empty_like(X)
    for j in range(X.shape[1]):
        y, info = spla.cg(M, X[:, j], rtol=rtol, atol=0.0, maxiter=5000)
        if info != 0:
            raise RuntimeError("oracle CG did not converge")
        out[:, j] = y
    return s * out


def phi_apply(A, mu, kind, param, X, **kw):
    if kind == "res":
        return phi_res_apply(A, mu, param, X, **kw)
    return phi_exp_apply(A, mu, param, X, **kw)


def fdeg(A, mu, kind, param, **kw):
    return phi_apply(A, mu, kind, param, np.ones((A.shape[0], 1)), **kw)[:, 0]


def apply_laplacian(A, mu, kind, param, X, w=None, **kw):
    if w is None:
        w = fdeg(A, mu, kind, param, **kw)
    return w[:, None] * X - phi_apply(A, mu, kind, param, X, **kw)
