"""Pins of the oracle's diffusion, sparse routes, estimators, Philox and MLP."""

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import estimators, genfun, laplacian, mlp, philox, sparse, walks


def er(n=60, m=150, seed=3):
    rp, ci = synth.erdos_renyi_gnm(n, m, seed)
    return n, rp, ci


# ------------------------------------------------------------------ diffusion
@pytest.mark.parametrize("t", [0.1, 1.0, 10.0])
def test_expv_matches_library_expm(t):
    n, rp, ci = er()
    A = walks.adjacency(n, rp, ci)
    L = laplacian.walk_laplacian(genfun.phi(A, 0.5, "exp", 1.0 / np.linalg.eigvalsh(A)[-1]))
    U0 = synth.gaussian_block(n, 3, 4)
    (Y,) = laplacian.expv(L, U0, [t])
    np.testing.assert_allclose(Y, sla.expm(-t * L) @ U0, atol=1e-11)


def test_diffusion_conserves_mass_and_positivity():
    """1^T exp(-tL) u = 1^T u (L 1 = 0, L symmetric); entries stay >= 0 for an
    M-matrix L (Sec. 2.1 discussion of the maximum principle)."""
    n, rp, ci = er()
    A = walks.adjacency(n, rp, ci)
    L = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))))
    u = synth.spike_block(n, [0, 7])
    for t, Y in zip([0.5, 5.0, 50.0], laplacian.expv(L, u, [0.5, 5.0, 50.0])):
        np.testing.assert_allclose(Y.sum(0), u.sum(0), atol=1e-12)
        assert Y.min() > -1e-12


def test_average_return_probability_limits():
    """p_hat(0) = 1 and p_hat(t) -> (number of components) / n."""
    rp, ci = synth.csr_from_edges(10, [0, 1, 2, 3, 5, 6, 7, 8], [1, 2, 3, 4, 6, 7, 8, 9])  # two paths
    A = walks.adjacency(10, rp, ci)
    L = laplacian.walk_laplacian(genfun.phi(A, 0.0, "exp", 0.5))
    assert abs(laplacian.average_return_probability(L, 0.0) - 1.0) < 1e-14
    assert abs(laplacian.average_return_probability(L, 1e4) - 2 / 10) < 1e-10


# ------------------------------------------------------------------ sparse routes
@pytest.mark.parametrize("mu", [0.0, 0.4, 1.0])
@pytest.mark.parametrize("kind", ["res", "exp"])
def test_sparse_routes_match_dense(mu, kind):
    n, rp, ci = er(200, 700, 9)
    Ad = walks.adjacency(n, rp, ci)
    As = sparse.adjacency(n, rp, ci)
    if kind == "res":
        param = 0.5 / sparse.rho_Z(As, mu)
    else:
        param = 1.0 / sparse.lambda_max(As)
    X = synth.gaussian_block(n, 5, 1)
    ph = genfun.phi(Ad, mu, kind, param)
    np.testing.assert_allclose(sparse.phi_apply(As, mu, kind, param, X), ph @ X, atol=1e-12 * np.abs(ph @ X).max())
    np.testing.assert_allclose(sparse.fdeg(As, mu, kind, param), ph.sum(1), rtol=1e-12)
    np.testing.assert_allclose(sparse.apply_laplacian(As, mu, kind, param, X), laplacian.apply_laplacian(ph, X),
                               atol=1e-11 * np.abs(ph @ X).max())


def test_sparse_rho_z_matches_dense():
    n, rp, ci = er(700, 2800, 2)  # large enough for the ARPACK branch
    As = sparse.adjacency(n, rp, ci)
    Ad = walks.adjacency(n, rp, ci)
    for mu in (0.0, 0.5, 1.0):
        dense = walks.spectral_radius(walks.linearisation(Ad, mu))
        assert abs(sparse.rho_Z(As, mu) - dense) < 1e-9 * dense


def test_rho_z_is_where_deformed_laplacian_becomes_singular():
    """det(lambda^2 I - lambda A + mu (D - mu I)) = 0  <=>  A_mu(1/lambda) singular,
    so the smallest eigenvalue of A_mu(t) crosses zero at t = 1/rho(Z)."""
    n, rp, ci = er(80, 240, 5)
    A = walks.adjacency(n, rp, ci)
    for mu in (0.25, 1.0):
        rho = walks.spectral_radius(walks.linearisation(A, mu))
        lmin = lambda t: np.linalg.eigvalsh(genfun.deformed_laplacian(A, mu, t))[0]
        assert abs(lmin(1.0 / rho)) < 1e-10
        assert lmin(0.99 / rho) > 0 and lmin(1.01 / rho) < 0


# ------------------------------------------------------------------ estimators
def low_rank_psd(n, r, seed):
    G = synth.gaussian_block(n, r, seed)
    return G @ G.T


def test_xnys_exact_for_rank_below_probe_count():
    n, r, M = 50, 5, 8
    F = low_rank_psd(n, r, 1)
    Om = philox.gaussian(n, M, 77)
    t, e, d, de = estimators.xnys(Om, F @ Om, rcond=1e-12)
    assert abs(t - np.trace(F)) < 1e-9 * np.trace(F)
    assert e < 1e-8 * np.trace(F)
    np.testing.assert_allclose(d, np.diag(F), atol=1e-9 * np.trace(F))


def test_control_variate_exact_for_diagonal_target():
    n, M = 30, 4
    F = np.diag(np.linspace(1, 3, n))
    Om = philox.gaussian(n, M, 3)
    np.testing.assert_allclose(estimators.cv_diag(Om, F @ Om, np.diag(F)), np.diag(F), atol=1e-14)
    np.testing.assert_allclose(estimators.bks_diag(Om, F @ Om), np.diag(F), atol=1e-14)


def test_hutchinson_unbiased_and_variance():
    """E[omega_i (F omega)_i] = F_ii; Var = 2 F_ii^2 + sum_{k != i} F_ik^2 for Gaussian omega."""
    n = 6
    F = low_rank_psd(n, 6, 2) + np.eye(n)
    M, reps = 8, 4000
    Om = philox.gaussian(n, M * reps, 123)
    Y = F @ Om
    est = (Om * Y).reshape(n, reps, M).mean(axis=2)
    var_pred = (2 * np.diag(F) ** 2 + (F ** 2).sum(1) - np.diag(F) ** 2) / M
    mean_err = np.abs(est.mean(1) - np.diag(F)) / np.sqrt(var_pred / reps)
    assert mean_err.max() < 4.5
    np.testing.assert_allclose(est.var(1, ddof=1), var_pred, rtol=0.12)


def test_xnys_trace_unbiased_on_full_rank():
    n, M, reps = 40, 6, 300
    F = low_rank_psd(n, n, 5) / n + 0.1 * np.eye(n)
    ts = []
    for s in range(reps):
        Om = philox.gaussian(n, M, 1000 + s)
        ts.append(estimators.xnys(Om, F @ Om)[0])
    ts = np.array(ts)
    assert abs(ts.mean() - np.trace(F)) < 4.5 * ts.std(ddof=1) / np.sqrt(reps)


def brute_triangles(A):
    n = A.shape[0]
    t = np.zeros(n)
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                if A[i, j] and A[j, k] and A[i, k]:
                    t[[i, j, k]] += 1
    return t


@pytest.mark.parametrize("mu", [0.0, 0.3, 1.0])
@pytest.mark.parametrize("kind", ["exp", "res"])
def test_low_order_series_diagonal_closed_form(mu, kind):
    """diag of sum_{k<=3} c_k q_k = 1 + c_2 (1 - mu) d + 2 c_3 t (t: triangles, counted
    by brute force over node triples; q_k from walk enumeration)."""
    n, rp, ci = er(25, 70, 8)
    A = walks.adjacency(n, rp, ci)
    c = genfun.coefficients(kind, 0.2, 3)
    G = genfun.phi_series(A, mu, c)
    d = A.sum(1)
    t = brute_triangles(A)
    assert t.sum() > 0
    np.testing.assert_allclose(np.diag(G), 1 + c[2] * (1 - mu) * d + 2 * c[3] * t, rtol=1e-14)


def test_surrogate_exact_when_target_is_the_surrogate():
    """F = G with Rademacher probes: omega_i^2 = 1 and the off-diagonal noise is gone,
    so the estimate is diag G for any control variate."""
    n, rp, ci = er(30, 80, 4)
    A = walks.adjacency(n, rp, ci)
    G = genfun.phi_series(A, 0.5, genfun.coefficients("exp", 0.3, 3))
    Om = philox.rademacher(n, 5, 9)
    Z = G @ Om
    np.testing.assert_allclose(estimators.surrogate_diag(Om, Z, Z, np.diag(G)), np.diag(G), rtol=1e-14)
    g = np.linspace(0.5, 2.0, n)
    np.testing.assert_allclose(estimators.surrogate_diag(Om, Z, Z, np.diag(G), g), np.diag(G), rtol=1e-14)
    assert abs(estimators.surrogate_trace(Om, Z, Z, np.diag(G)) - np.trace(G)) < 1e-12 * np.trace(G)


def test_surrogate_unbiased_and_removes_offdiagonal_noise():
    """E[d_hat] = diag F for any g; the per-node variance is that of Hutchinson on F - G
    (Gaussian: 2 (F_ii - g_i)^2 + sum_{k != i} (F - G)_ik^2), below plain Hutchinson."""
    n = 8
    rp, ci = synth.erdos_renyi_gnm(n, 14, 2)
    A = walks.adjacency(n, rp, ci)
    F = genfun.phi(A, 0.5, "exp", 0.4)
    G = genfun.phi_series(A, 0.5, genfun.coefficients("exp", 0.4, 3))
    g = np.diag(F) * 1.1
    M, reps = 4, 4000
    Om = philox.gaussian(n, M * reps, 31)
    Y, Z = F @ Om, G @ Om
    est = np.stack([estimators.surrogate_diag(Om[:, r * M:(r + 1) * M], Y[:, r * M:(r + 1) * M],
                                              Z[:, r * M:(r + 1) * M], np.diag(G), g) for r in range(reps)], 1)
    R = F - G
    var_pred = (2 * (np.diag(F) - g) ** 2 + (R ** 2).sum(1) - np.diag(R) ** 2) / M
    z = np.abs(est.mean(1) - np.diag(F)) / np.sqrt(var_pred / reps)
    assert z.max() < 4.5
    np.testing.assert_allclose(est.var(1, ddof=1), var_pred, rtol=0.15)
    var_plain = (2 * np.diag(F) ** 2 + (F ** 2).sum(1) - np.diag(F) ** 2) / M
    assert np.all(var_pred < var_plain)


# ------------------------------------------------------------------ philox
def test_philox_known_answer_vectors():
    """Published Philox4x32-10 known-answer vectors (Random123 distribution)."""
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
        ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
        ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
         [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
    ]
    for c, k, out in kat:
        got = philox.philox4x32_10(np.array(c, dtype=np.uint64), np.array(k, dtype=np.uint64))
        assert [int(x) for x in got] == out


def test_probe_laws():
    g = philox.gaussian(4000, 16, 9)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1) < 0.01
    r = philox.rademacher(4000, 16, 9)
    assert set(np.unique(r)) == {-1.0, 1.0} and abs(r.mean()) < 0.02


# ------------------------------------------------------------------ MLP
def test_mlp_gradient_finite_differences():
    p = synth.glorot_params(mlp.SIZES, 1)
    X = synth.gaussian_block(20, 8, 2)
    t = synth.gaussian_block(20, 1, 3)[:, 0]
    L, g = mlp.loss_and_grad(p, X, t)
    rng = np.random.default_rng(0)
    for idx in rng.choice(mlp.NPARAM, 40, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[idx] += h
        pm[idx] -= h
        fd = (mlp.loss_and_grad(pp, X, t)[0] - mlp.loss_and_grad(pm, X, t)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-7 * max(1.0, abs(g[idx])), idx


def test_mlp_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    p = synth.glorot_params(mlp.SIZES, 4)
    X = synth.gaussian_block(33, 8, 5)
    t = synth.gaussian_block(33, 1, 6)[:, 0]
    L, g = mlp.loss_and_grad(p, X, t)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    parts, o = [], 0
    for s in mlp.SIZES:
        k = int(np.prod(s))
        parts.append(pt[o:o + k].reshape(s))
        o += k
    W1, b1, W2, b2, W3, b3 = parts
    Xt = torch.tensor(X)
    y = torch.tanh(torch.tanh(Xt @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    loss = ((y[:, 0] - torch.tensor(t)) ** 2).mean()
    loss.backward()
    assert abs(loss.item() - L) < 1e-14
    np.testing.assert_allclose(pt.grad.numpy(), g, atol=1e-14)


def test_adam_first_step_is_signed_lr():
    p = np.zeros(5)
    g = np.array([1.0, -2.0, 0.5, -0.1, 3.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(5), np.zeros(5), 1, 0.01)
    np.testing.assert_allclose(p1, -0.01 * np.sign(g), rtol=1e-6)
