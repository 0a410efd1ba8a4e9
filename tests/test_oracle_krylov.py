"""Pins of the same-K block Krylov reference (oracle.krylov): exhaustion of the space
reproduces the dense functions, exactness for low-degree polynomials (and not beyond),
the block Lanczos decomposition, the row-chunked sparse product, and the diffusion's
outer Lanczos against dense eigendecompositions."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import genfun, krylov, laplacian, walks


def graph(n, m, seed):
    rp, ci = synth.erdos_renyi_gnm(n, m, seed)
    A = walks.adjacency(n, rp, ci)
    return A, sp.csr_matrix(A)


@pytest.mark.parametrize("reorth", ["full", "local"])
def test_exhausted_space_gives_dense_resolvent_and_exponential(reorth):
    """K b >= n: the block Krylov space is R^n and the approximation is exact."""
    n, b = 40, 4
    A, As = graph(n, 120, 3)
    lam = np.linalg.eigvalsh(A)[-1]
    X = synth.gaussian_block(n, b, 4)
    K = n // b + 1
    for mu in (0.0, 0.5, 1.0):
        alpha = 0.5 / walks.spectral_radius(walks.linearisation(A, mu))
        ref = genfun.phi(A, mu, "res", alpha) @ X
        got = krylov.phi_resolvent_lanczos(As, mu, alpha, X, K, reorth="full")
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11, mu
    ref = genfun.phi(A, 0.0, "exp", 1.0 / lam) @ X
    got = krylov.phi_exp_lanczos(As, 1.0 / lam, X, K, reorth="full")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-11
    if reorth == "local":
        # with K b < n / 2 the local policy keeps the basis orthonormal to rounding
        K = 3
        Y, (V, _, _, _) = krylov.lanczos_function(lambda Z: As @ Z, X, K, lambda x: x, reorth="local")
        Vm = np.hstack(V[:K])
        assert np.abs(Vm.T @ Vm - np.eye(K * b)).max() < 1e-12


def test_polynomial_exactness_and_its_limit():
    """K block Lanczos steps reproduce p(A) X exactly for deg p <= K - 1, since
    A^k X lies in the span of V_0 .. V_{K-1}; degree 2K is not reproduced."""
    n, b, K = 300, 2, 6
    _, As = graph(n, 1200, 7)
    X = synth.gaussian_block(n, b, 8)
    Ad = As.toarray()
    ref = np.linalg.matrix_power(Ad, K - 1) @ X
    got, _ = krylov.lanczos_function(lambda Z: As @ Z, X, K, lambda x: x ** (K - 1), reorth="full")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-12
    ref = np.linalg.matrix_power(Ad, 2 * K) @ X
    got, _ = krylov.lanczos_function(lambda Z: As @ Z, X, K, lambda x: x ** (2 * K), reorth="full")
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) > 1e-6


def test_block_lanczos_decomposition():
    """Op [V_0 .. V_{K-1}] = [V_0 .. V_{K-1}] T + V_K B_{K-1} E_K^T, V orthonormal,
    X = V_0 R_0."""
    n, b, K = 500, 3, 8
    _, As = graph(n, 2500, 11)
    d = np.asarray(As.sum(1)).ravel()
    mu, alpha = 0.5, 0.05
    op = krylov.deformed_apply(As, mu, alpha)
    X = synth.gaussian_block(n, b, 12)
    V, A, B, R0 = krylov.block_lanczos(op, X, K, reorth="local")
    Vm = np.hstack(V[:K])
    T = krylov.block_tridiagonal(A, B)
    lhs = op(Vm)
    rhs = Vm @ T
    rhs[:, (K - 1) * b:] += V[K] @ B[K - 1]
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()
    assert np.abs(Vm.T @ Vm - np.eye(K * b)).max() < 1e-12
    assert np.abs(V[0] @ R0 - X).max() < 1e-13 * np.abs(X).max()
    # the operator itself is eq. deformed
    M = (1 - mu * mu * alpha * alpha) * np.eye(n) - alpha * As.toarray() + alpha * alpha * mu * np.diag(d)
    assert np.abs(op(X) - M @ X).max() < 1e-13


def test_threaded_spmm_is_the_plain_product():
    rp, ci = synth.barabasi_albert(20000, 3, 5)
    n = len(rp) - 1
    As = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    X = synth.gaussian_block(n, 5, 6)
    assert np.array_equal(krylov.spmm(As, X), As @ X)


def test_series_matches_dense_series():
    n = 60
    A, As = graph(n, 200, 13)
    X = synth.gaussian_block(n, 3, 14)
    c = krylov.exp_coefficients(0.2, 9)
    for mu in (0.0, 0.3, 1.0):
        np.testing.assert_allclose(krylov.series_apply(As, mu, c, X), genfun.phi_series(A, mu, c) @ X, rtol=1e-12,
                                   atol=1e-12)


def test_expv_outer_lanczos_against_dense():
    """Outer Lanczos on L with the inner series: exhausted space gives the dense
    exp(-t L) of the same (truncated) phi; a short space converges towards it and its
    a-posteriori estimate has the order of the true error."""
    n, b = 48, 4
    A, As = graph(n, 150, 21)
    lam = np.linalg.eigvalsh(A)[-1]
    mu, beta, Kin = 0.5, 1.0 / lam, 12
    c = krylov.exp_coefficients(beta, Kin)
    phi = genfun.phi_series(A, mu, c)
    w = phi.sum(1)
    U0 = synth.gaussian_block(n, b, 22)
    ts = [0.1, 1.0, 10.0]
    refs = laplacian.expv(laplacian.walk_laplacian(phi), U0, ts)
    Ys, errs = krylov.expv_lanczos(lambda X: krylov.series_apply(As, mu, c, X), w, U0, ts, n // b + 1)
    for y, r in zip(Ys, refs):
        assert np.linalg.norm(y - r) / np.linalg.norm(r) < 1e-11
    # a larger graph, shorter space: error decreases with K; the estimate tracks it
    n = 400
    A, As = graph(n, 1600, 23)
    lam = np.linalg.eigvalsh(A)[-1]
    c = krylov.exp_coefficients(1.0 / lam, 14)
    phi = genfun.phi_series(A, mu, c)
    U0 = synth.gaussian_block(n, b, 24)
    (ref,) = laplacian.expv(laplacian.walk_laplacian(phi), U0, [1.0])
    prev = np.inf
    for K in (3, 6, 10):
        (y,), (est,) = krylov.expv_lanczos(lambda X: krylov.series_apply(As, mu, c, X), phi.sum(1), U0, [1.0], K)
        err = np.linalg.norm(y - ref)
        assert err < prev
        assert est / 100 < err < est * 100 or err < 1e-12, (K, err, est)
        prev = err
