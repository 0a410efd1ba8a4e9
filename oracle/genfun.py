"""Generating functions phi(A, c) = sum_k c_k q_k(A), dense float64 (Sec. 3.2.1).

Two weight families are used by the paper:
  * resolvent  c_k = alpha^k            (Sec. 3.2.1, eq. deformed and the
    resolvent NBT Laplacian paragraph);
  * exponential c_k = beta^k / k!       (exponential NBT paragraph; beta is the
    "inverse temperature" of Sec. 4.1.2).
c_0 = 1 in both.  Reading: the walk degree w = phi 1 keeps the c_0 term (it
cancels in the Laplacian but not in w); the paper's Fig. 1 stationary
distributions reproduce only with c_0 included.

phi is computed by three independent dense routes, which the tests require to
agree:
  1. the truncated series (definition, Prop. "whe-we-converge");
  2. the linearisation  phi = [I O] f_1(Z) [q_1; q_2] + c_0 I  (same
     proposition, second identity);
  3. for the resolvent, the closed form  phi = (1 - mu^2 a^2) A_mu(a)^{-1}
     with A_mu(a) = (1 - mu^2 a^2) I - a A + a^2 mu D.  This is eq. deformed
     (mu = 1) extended to every mu in [0, 1], as the remark after
     Prop. "CGworks" states; derived by summing the recurrence eq. qrec against
     x^k.
Test infrastructure: see the package docstring.
"""

import math

import numpy as np
import scipy.linalg as sla

from .walks import btdw_counts, degrees, linearisation

RESOLVENT = "res"
EXPONENTIAL = "exp"


def coefficients(kind, param, kmax):
    """c_0 .. c_kmax for the two weight families."""
    if kind == RESOLVENT:
        return np.array([param ** k for k in range(kmax + 1)], dtype=np.float64)
    if kind == EXPONENTIAL:
        return np.array([param ** k / math.factorial(k) for k in range(kmax + 1)], dtype=np.float64)
    raise ValueError(kind)


def phi_series(A, mu, coeffs):
    """Truncated definition sum_{k<=K} c_k q_k(A) (Prop. "whe-we-converge")."""
    q = btdw_counts(A, mu, len(coeffs) - 1)
    out = np.zeros_like(A)
    for ck, qk in zip(coeffs, q):
        out += ck * qk
    return out


def deformed_laplacian(A, mu, alpha):
    """A_mu(alpha) = (1 - mu^2 alpha^2) I - alpha A + alpha^2 mu D.
    At mu = 1 this is I - alpha A - alpha^2 (I - D) (eq. deformed)."""
    n = A.shape[0]
    return (1.0 - mu * mu * alpha * alpha) * np.eye(n) - alpha * A + alpha * alpha * mu * np.diag(degrees(A))


def phi_resolvent_closed(A, mu, alpha):
    """Closed form of the resolvent generating function (eq. deformed, general mu)."""
    n = A.shape[0]
    return (1.0 - mu * mu * alpha * alpha) * np.linalg.solve(deformed_laplacian(A, mu, alpha), np.eye(n))


def _q12(A, mu):
    q = btdw_counts(A, mu, 2)
    return np.vstack([q[1], q[2]])


def phi_resolvent_linearised(A, mu, alpha):
    """[I O] f_1(Z) [q_1; q_2] + I with f_1(x) = sum_k alpha^{k+1} x^k = alpha / (1 - alpha x)."""
    n = A.shape[0]
    Z = linearisation(A, mu)
    F = alpha * np.linalg.solve(np.eye(2 * n) - alpha * Z, _q12(A, mu))
    return F[:n] + np.eye(n)


def phi1_times(M, B):
    """phi_1(M) B with phi_1(x) = (e^x - 1)/x, read off the top-right block of
    expm([[M, B], [0, 0]]) (a standard identity for the first phi-function)."""
    m, k = B.shape
    aug = np.zeros((m + k, m + k))
    aug[:m, :m] = M
    aug[:m, m:] = B
    return sla.expm(aug)[:m, m:]


def phi_exponential_linearised(A, mu, beta, selector="I O"):
    """Exponential weights via the linearisation (Prop. "whe-we-converge",
    Cor. "when-we-converge"):  phi = [I O] f_1(Z) [q_1; q_2] + I, where for
    c_k = beta^k / k! one has f_1(x) = sum_k beta^{k+1} x^k / (k+1)! = beta phi_1(beta x).

    ``selector="O I"`` evaluates [O I] f_1(Z) [q_1; q_2] instead (no "+ I").
    That is the reading under which the paper's Fig. 1 bar for the exponential
    NBT Laplacian is reproduced; the displayed formula eq. exp-based-laplacian
    uses [I O].  Only the regression test of Fig. 1 uses it.
    """
    n = A.shape[0]
    Z = linearisation(A, mu)
    F = beta * phi1_times(beta * Z, _q12(A, mu))
    if selector == "I O":
        return F[:n] + np.eye(n)
    if selector == "O I":
        return F[n:]
    raise ValueError(selector)


def phi(A, mu, kind, param):
    """phi(A, c) for the resolvent (closed form) or the exponential (linearisation)."""
    if kind == RESOLVENT:
        return phi_resolvent_closed(A, mu, param)
    if kind == EXPONENTIAL:
        return phi_exponential_linearised(A, mu, param)
    raise ValueError(kind)


def exp_tail_bound(beta, lam, K):
    """Bound on || sum_{k>K} c_k q_k ||_2 for c_k = beta^k/k!: since 0 <= q_k <= A^k
    entrywise (weights in [0, 1]), ||q_k||_2 <= lambda_max(A)^k."""
    x = beta * lam
    tot, term = 0.0, 1.0
    for k in range(1, K + 200):
        term *= x / k
        if k > K:
            tot += term
            if term < 1e-300 or term < 1e-18 * tot:
                break
    return tot
