"""The rational Krylov return-probability oracle (Alg. 1, Sec. 4.4) against facts fixed
by the mathematics.

Pins: AAA recovers the poles of a rational function exactly and approximates exp(-x)
to its tolerance between the sample points; a constant has no poles; the block
rational Arnoldi decomposition L V K = V H holds with orthonormal V; the space
contains (L - xi)^{-1} Omega for every finite pole xi (the definition of the space,
eq. block-rational-Krylov); with a closing infinite pole the reduced pencil is the
Rayleigh quotient V_k^H L V_k; once the basis spans everything Alg. 1 returns the
Nystrom estimate of the exact exp(-t L) Omega; on a graph with c components p(t)
tends to c / n, which the estimator reproduces exactly (rank-c target, M > c)."""

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import estimators, genfun, laplacian, rational, walks


def walk_lap(n, m, seed, mu=0.5, kind="exp", p=None):
    rp, ci = synth.barabasi_albert(n, m, seed=seed)
    A = walks.adjacency(n, rp, ci)
    if p is None:
        p = 1.0 / np.linalg.eigvalsh(A).max()
    return laplacian.walk_laplacian(genfun.phi(A, mu, kind, p))


def test_aaa_recovers_poles_of_a_rational_function():
    Z = np.linspace(0.0, 10.0, 2000)
    F = 1.0 / (Z + 1.0) + 2.0 / ((Z - 3.0) ** 2 + 1.0)
    z, f, w, poles, err = rational.aaa(F, Z)
    assert err < 1e-13
    want = np.array([-1.0, 3.0 - 1.0j, 3.0 + 1.0j])
    got = np.sort_complex(poles)
    assert got.size == 3
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-9)


def test_aaa_constant_has_no_poles():
    Z = np.linspace(0.0, 1.0, 50)
    _, _, _, poles, err = rational.aaa(np.full(50, 2.5), Z)
    assert err < 1e-14 and poles.size == 0


@pytest.mark.parametrize("xmax", [10.0, 300.0, 1000.0])
def test_aaa_exp_between_sample_points(xmax):
    Z = rational.exp_sample_points(xmax)
    z, f, w, poles, err = rational.aaa(np.exp(-Z), Z)
    x = np.linspace(0.0, xmax, 30011)   # mostly not sample points
    r = rational.aaa_eval(z, f, w, x)
    assert np.abs(r - np.exp(-x)).max() < 1e-11
    assert np.abs(r.imag).max() < 1e-12
    # real data: poles closed under conjugation, none on the interval
    gap = np.abs(poles[:, None] - poles.conj()[None, :]).min(axis=1)
    assert gap.max() < 1e-6 * xmax
    kept = rational.exp_poles(xmax)
    on = (np.abs(kept.imag) < 1e-8 * xmax) & (kept.real >= 0) & (kept.real <= xmax)
    assert not on.any() and kept.size >= poles.size - 2


def test_rational_arnoldi_decomposition_and_space():
    Lap = walk_lap(60, 2, seed=3)
    n, M = 60, 3
    Om = synth.gaussian_block(n, M, seed=4)
    poles = [-1.0, 2.0 + 1.5j, 2.0 - 1.5j, np.inf, -0.3]
    V, K, H, R0 = rational.rational_arnoldi(Lap, Om, poles)
    assert V.shape == (n, (len(poles) + 1) * M)
    np.testing.assert_allclose(V.conj().T @ V, np.eye(V.shape[1]), atol=1e-12)
    np.testing.assert_allclose(V[:, :M] @ R0, Om, atol=1e-12)
    res = Lap @ V @ K - V @ H
    assert np.linalg.norm(res) < 1e-11 * np.linalg.norm(Lap) * np.linalg.norm(K)
    # (L - xi)^{-1} Omega lies in the space for every finite pole
    P = V @ V.conj().T
    for xi in poles:
        if np.isinf(xi):
            continue
        X = np.linalg.solve(Lap - xi * np.eye(n), Om)
        assert np.linalg.norm(X - P @ X) < 1e-10 * np.linalg.norm(X)
    # a pole sign error would put the other shift in the space instead
    X = np.linalg.solve(Lap + 2.0 * np.eye(n), Om)
    assert np.linalg.norm(X - P @ X) > 1e-6 * np.linalg.norm(X)


def test_reduced_pencil_is_rayleigh_quotient_with_closing_infinite_pole():
    Lap = walk_lap(50, 2, seed=8, mu=1.0, kind="res", p=0.1)
    n, M = 50, 2
    Om = synth.gaussian_block(n, M, seed=9)
    seq = [-0.5, 1.0 + 2.0j, 1.0 - 2.0j, np.inf]
    V, K, H, _ = rational.rational_arnoldi(Lap, Om, seq)
    Ak = rational.reduced_pencil_matrix(K, H, M)
    Vk = V[:, :len(seq) * M]
    np.testing.assert_allclose(Ak, Vk.conj().T @ Lap @ Vk, atol=1e-11 * np.linalg.norm(Lap))


def test_full_space_gives_nystrom_of_exact_exponential():
    Lap = walk_lap(12, 2, seed=1)
    n, M = 12, 3
    Om = synth.gaussian_block(n, M, seed=2)
    ts = [0.5, 5.0]
    poles = np.array([-1.0, 1.5 + 1.0j, 1.5 - 1.0j])   # with the closing inf: 4 blocks of 3 span R^12
    p, e, _ = rational.return_probability_estimate(Lap, Om, ts, 10.0, 1.0, poles=poles)
    lam, S = np.linalg.eigh(Lap)
    for t, pt, et in zip(ts, p, e):
        Y = S @ (np.exp(-t * lam)[:, None] * (S.T @ Om)) / n
        tr, te, _, _ = estimators.xnys(Om, Y)
        assert abs(pt - tr) < 1e-10 * abs(tr)
        assert abs(et - te) < 1e-8 * max(te, 1e-300) + 1e-14


def test_components_limit():
    # three components (Barabasi-Albert graphs of 40 nodes); L's null space has dimension 3
    blocks = []
    for seed in (1, 2, 3):
        rp, ci = synth.barabasi_albert(40, 2, seed=seed)
        blocks.append(walks.adjacency(40, rp, ci))
    A = sla.block_diag(*blocks)
    n = A.shape[0]
    Lap = laplacian.walk_laplacian(genfun.phi(A, 0.0, "exp", 0.1))
    Om = synth.gaussian_block(n, 5, seed=6)
    rho = np.linalg.eigvalsh(Lap).max()
    t_end = 200.0 / np.sort(np.linalg.eigvalsh(Lap))[3]     # exp(-t lambda_4) = e^-200
    p, e, _ = rational.return_probability_estimate(Lap, Om, [t_end], t_end, rho, pole_time=t_end)
    assert abs(p[0] - 3.0 / n) < 1e-9
    assert e[0] < 1e-9
    np.testing.assert_allclose(rational.exact_return_probability(Lap, [t_end]), [3.0 / n], atol=1e-12)


def test_pole_placement_accuracy():
    """AAA poles of exp(-x) on [0, t* rho]: used as printed they approximate exp(-t L)
    Omega well for t near 1; divided by t* they do so for t near t*."""
    Lap = walk_lap(300, 2, seed=5, mu=0.5)
    n, M, tmax = 300, 4, 100.0
    Om = synth.gaussian_block(n, M, seed=1)
    lam, S = np.linalg.eigh(Lap)
    rho = lam.max()
    polesx = rational.exp_poles(tmax * rho)

    def rel_err(poles, t):
        seq = list(poles) + [np.inf]
        V, K, H, _ = rational.rational_arnoldi(Lap, Om, seq)
        Ak = rational.reduced_pencil_matrix(K, H, M)
        Vk = V[:, :len(seq) * M]
        Y = (Vk @ (sla.expm(-t * Ak) @ (Vk.conj().T @ Om))).real
        Ye = S @ (np.exp(-t * lam)[:, None] * (S.T @ Om))
        return np.linalg.norm(Y - Ye) / np.linalg.norm(Ye)

    assert rel_err(polesx, 1.0) < 1e-8
    assert rel_err(polesx / tmax, tmax) < 1e-8
