"""Rational Krylov estimate of the average return probability (Alg. 1, Sec. 4.4), float64.

Test infrastructure: see the package docstring.

* AAA (Nakatsukasa, Sete, Trefethen, SIAM J. Sci. Comput. 2018; the pole
  construction cited in Alg. 1): greedy barycentric rational approximation of
  samples F on points Z; weights from the last right singular vector of the Loewner
  matrix over the points not yet chosen; poles are the finite eigenvalues of the
  arrowhead pencil of the barycentric denominator.
* Block rational Arnoldi (eq. block-rational-Krylov and the decomposition
  L V_{k+1} K_k = V_{k+1} H_k): complex arithmetic, exact dense solves, each new
  block built from the last basis block (continuation) and orthogonalised twice
  against the whole basis.
* Alg. 1: Y(t) = (1/n) V_k exp(-t Hhat Khat^{-1}) V_k^H Omega on the reduced pencil,
  then the leave-one-out Nystrom estimator on (Y(t), Omega).

Readings where the paper is silent: the AAA poles of exp(-x) on [0, t* rho(L)] serve
as poles of the space as they are (pole_time = 1, the text of Alg. 1), or divided by
a time tau (pole_time = tau: the poles of r(tau lambda) ~ exp(-tau lambda), which
target t near tau); the pole sequence is closed by one infinite pole, so the reduced
pencil is the Rayleigh quotient of L on the first k blocks.
"""

import numpy as np
import scipy.linalg as sla

from . import estimators


def aaa(F, Z, tol=1e-13, mmax=100):
    """AAA on samples F = f(Z).  Returns (support points z, values f, weights w,
    poles, max error on Z)."""
    Z = np.asarray(Z, dtype=np.complex128)
    F = np.asarray(F, dtype=np.complex128)
    M = Z.size
    J = np.ones(M, dtype=bool)        # points not (yet) chosen as support points
    zs, fs = [], []
    C = np.zeros((M, 0), dtype=np.complex128)
    R = np.full(M, F.mean())
    w = np.zeros(0)
    err = np.inf
    scale = np.abs(F).max()
    for _ in range(mmax):
        j = int(np.argmax(np.where(J, np.abs(F - R), -1.0)))
        zs.append(Z[j])
        fs.append(F[j])
        J[j] = False
        col = np.zeros(M, dtype=np.complex128)
        col[J] = 1.0 / (Z[J] - Z[j])
        C = np.column_stack([C, col])
        fz = np.array(fs)
        A = F[J, None] * C[J] - C[J] * fz[None, :]     # Loewner matrix on the free points
        _, _, Vh = np.linalg.svd(A, full_matrices=False)
        w = Vh[-1].conj()
        N = C @ (w * fz)
        D = C @ w
        R = F.copy()
        R[J] = N[J] / D[J]
        err = np.abs(F - R).max()
        if err <= tol * scale:
            break
    z = np.array(zs)
    f = np.array(fs)
    m = z.size
    # poles: the finite eigenvalues of the pencil (E, B), E = [[0, w^T], [1, diag z]]
    E = np.zeros((m + 1, m + 1), dtype=np.complex128)
    E[0, 1:] = w
    E[1:, 0] = 1.0
    E[1:, 1:] = np.diag(z)
    B = np.eye(m + 1, dtype=np.complex128)
    B[0, 0] = 0.0
    ev = sla.eig(E, B, right=False)
    poles = ev[np.isfinite(ev)]
    return z, f, w, poles, float(err)


def aaa_eval(z, f, w, x):
    """The barycentric approximant r(x) = sum w_j f_j / (x - z_j) / sum w_j / (x - z_j)."""
    x = np.asarray(x, dtype=np.complex128)
    out = np.empty(x.shape, dtype=np.complex128)
    for i, xi in enumerate(x.ravel()):
        d = xi - z
        hit = np.nonzero(d == 0)[0]
        if hit.size:
            out.ravel()[i] = f[hit[0]]
        else:
            c = w / d
            out.ravel()[i] = (c @ f) / c.sum()
    return out


def exp_sample_points(xmax, count=1000):
    """Points on [0, xmax] where exp(-x) is sampled: equispaced ones plus ones
    geometrically graded towards 0 (where exp(-x) varies most in relative terms)."""
    lin = np.linspace(0.0, xmax, count)
    geo = xmax * np.logspace(-6, 0, count)
    return np.unique(np.concatenate([lin, geo]))


def exp_poles(xmax, tol=1e-13, mmax=100):
    """AAA poles of exp(-x) on [0, xmax] (Alg. 1, pole construction).  Real poles on
    the interval itself are dropped: they are spurious pole-zero pairs of AAA (the
    approximant stays accurate between the sample points) and cannot serve as shifts
    of a matrix whose spectrum the interval covers."""
    Z = exp_sample_points(xmax)
    _, _, _, poles, _ = aaa(np.exp(-Z), Z, tol=tol, mmax=mmax)
    on = (np.abs(poles.imag) <= 1e-8 * xmax) & (poles.real >= 0.0) & (poles.real <= xmax)
    return poles[~on]


def _orth_block(V, W, passes=2):
    """Orthogonalise W against the columns of V twice (classical Gram-Schmidt), then
    QR.  Returns (coefficients against V, Q, R)."""
    c = np.zeros((V.shape[1], W.shape[1]), dtype=np.complex128)
    for _ in range(passes):
        if V.shape[1]:
            d = V.conj().T @ W
            W = W - V @ d
            c = c + d
    Q, R = np.linalg.qr(W)
    return c, Q, R


def rational_arnoldi(Lap, Omega, poles):
    """Block rational Arnoldi: V (n x (k+1)M, orthonormal columns), K, H ((k+1)M x kM)
    with Lap V K = V H.  A finite pole xi adds W = (Lap - xi I)^{-1} V_j, the pole
    inf adds W = Lap V_j, V_j being the last block (the continuation)."""
    n, M = Omega.shape
    k = len(poles)
    Lc = np.asarray(Lap, dtype=np.complex128)
    Q, R0 = np.linalg.qr(np.asarray(Omega, dtype=np.complex128))
    V = Q
    K = np.zeros(((k + 1) * M, k * M), dtype=np.complex128)
    H = np.zeros(((k + 1) * M, k * M), dtype=np.complex128)
    for j, xi in enumerate(poles):
        U = V[:, j * M:(j + 1) * M]
        if np.isinf(xi):
            W = Lc @ U
        else:
            W = np.linalg.solve(Lc - xi * np.eye(n), U)
        c, Qn, Rn = _orth_block(V, W)
        chat = np.vstack([c, Rn])            # W = V_{j+1} chat
        V = np.hstack([V, Qn])
        Ej = np.zeros(((j + 2) * M, M), dtype=np.complex128)
        Ej[j * M:(j + 1) * M] = np.eye(M)
        cols = slice(j * M, (j + 1) * M)
        if np.isinf(xi):
            # Lap V_j = V chat
            K[:(j + 2) * M, cols] = Ej
            H[:(j + 2) * M, cols] = chat
        else:
            # (Lap - xi) V chat = V_j  =>  Lap V chat = V (xi chat + E_j)
            K[:(j + 2) * M, cols] = chat
            H[:(j + 2) * M, cols] = xi * chat + Ej
    return V, K, H, R0


def reduced_pencil_matrix(K, H, M):
    """Hhat Khat^{-1}: the pencil without its last block row."""
    m = K.shape[1]
    return np.linalg.solve(K[:m].T, H[:m].T).T


def return_probability_estimate(Lap, Omega, ts, tmax, rho, tol=1e-13, rcond=1e-10, poles=None, pole_time=1.0):
    """Alg. 1: p_hat(t) and e_hat(t) for every t, from one rational Krylov basis.
    Poles: the AAA poles of exp(-x) on [0, tmax rho] divided by pole_time, closed by
    inf (or the given finite poles, closed by inf).  Returns (p_hat, e_hat, poles)."""
    n, M = Omega.shape
    if poles is None:
        poles = exp_poles(tmax * rho, tol=tol) / pole_time
    seq = list(poles) + [np.inf]
    V, K, H, _ = rational_arnoldi(Lap, Omega, seq)
    k = len(seq)
    Ak = reduced_pencil_matrix(K, H, M)
    Vk = V[:, :k * M]
    G = Vk.conj().T @ Omega
    p, e = [], []
    for t in ts:
        Y = (Vk @ (sla.expm(-t * Ak) @ G)).real / n
        tr, te, _, _ = estimators.xnys(Omega, Y, rcond=rcond)
        p.append(tr)
        e.append(te)
    return np.array(p), np.array(e), np.asarray(poles)


def exact_return_probability(Lap, ts):
    """p(t) = tr exp(-t L) / n (eq. average_return_probabilities), by eigh."""
    lam = np.linalg.eigvalsh(Lap)
    n = Lap.shape[0]
    return np.array([np.exp(-t * lam).sum() / n for t in ts])
