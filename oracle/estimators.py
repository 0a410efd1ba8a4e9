"""Stochastic diagonal and trace estimators (Sec. 4.4, Alg. 1), float64.

Inputs are the probe block Omega (n x M, columns omega_j) and Y = F Omega for a
symmetric target F (phi, or exp(-t L) for the return probabilities of Sec. 4.4).

* Hutchinson diagonal: d_i = (1/M) sum_j Omega_ij Y_ij.
* BKS-normalised diagonal: d_i = sum_j Omega_ij Y_ij / sum_j Omega_ij^2.
* Nystrom-type exchangeable estimator (the XNysTrace idea the paper adapts in
  Alg. 1): for each j, the Nystrom approximation built from the other probes,
      F_(j) = Y_{-j} (Omega_{-j}^T Y_{-j})^+ Y_{-j}^T,
  is corrected by the probe it left out:
      t_j = tr F_(j) + omega_j^T (F - F_(j)) omega_j,
      d_j = diag F_(j) + omega_j * (F - F_(j)) omega_j,
  and the estimates are the means over j, with error estimate std_j / sqrt(M).
  Written here literally, one j at a time.  The pseudo-inverse discards
  eigenvalues of the symmetrised core below rcond times its largest.
  The Nystrom approximation needs F positive semidefinite.
* Control-variate diagonal: with a prediction g of diag F,
      d_i = g_i + (1/M) sum_j Omega_ij (Y_ij - g_i Omega_ij).
* Low-order surrogate: with a matrix G whose diagonal is known exactly and
  Z = G Omega, Hutchinson on F - G plus diag G, optionally with a control variate g:
      d_i = g_i + (1/M) sum_j Omega_ij ((Y - Z)_ij + (diag G_i - g_i) Omega_ij),
  g = diag G when no control variate is given.  Only G's off-diagonal part is
  removed from the probe noise, so the estimator stays unbiased for any g.
Test infrastructure: see the package docstring.
"""

import numpy as np


def hutchinson_diag(Omega, Y):
    return (Omega * Y).mean(axis=1)


def hutchinson_trace(Omega, Y):
    return float((Omega * Y).sum() / Omega.shape[1])


def bks_diag(Omega, Y):
    return (Omega * Y).sum(axis=1) / (Omega * Omega).sum(axis=1)


def cv_diag(Omega, Y, g):
    g = np.asarray(g, dtype=np.float64)
    return g + (Omega * (Y - g[:, None] * Omega)).mean(axis=1)


def surrogate_diag(Omega, Y, Z, gdiag, g=None):
    gdiag = np.asarray(gdiag, dtype=np.float64)
    g = gdiag if g is None else np.asarray(g, dtype=np.float64)
    return g + (Omega * ((Y - Z) + (gdiag - g)[:, None] * Omega)).mean(axis=1)


def surrogate_trace(Omega, Y, Z, gdiag):
    """tr G + the mean over probes of omega_j^T (F - G) omega_j."""
    return float(np.sum(gdiag)) + float((Omega * (Y - Z)).sum() / Omega.shape[1])


def _pinv_sym(H, rcond):
    Hs = 0.5 * (H + H.T)
    lam, U = np.linalg.eigh(Hs)
    keep = lam > rcond * max(lam.max(), 0.0)
    inv = np.zeros_like(lam)
    inv[keep] = 1.0 / lam[keep]
    return (U * inv) @ U.T


def xnys(Omega, Y, rcond=1e-10):
    """Leave-one-out Nystrom estimator.  Returns (trace, trace_err, diag, diag_err)."""
    n, M = Omega.shape
    tr = np.empty(M)
    dg = np.empty((n, M))
    for j in range(M):
        keep = [k for k in range(M) if k != j]
        Om, Yk = Omega[:, keep], Y[:, keep]
        Hp = _pinv_sym(Om.T @ Yk, rcond)
        # F_(j) = Yk Hp Yk^T, never formed
        diag_hat = np.einsum("ik,kl,il->i", Yk, Hp, Yk)
        resid = Y[:, j] - Yk @ (Hp @ (Yk.T @ Omega[:, j]))
        tr[j] = diag_hat.sum() + Omega[:, j] @ resid
        dg[:, j] = diag_hat + Omega[:, j] * resid
    t = float(tr.mean())
    e = float(tr.std(ddof=1) / np.sqrt(M)) if M > 1 else float("inf")
    d = dg.mean(axis=1)
    de = dg.std(axis=1, ddof=1) / np.sqrt(M) if M > 1 else np.full(n, np.inf)
    return t, e, d, de
