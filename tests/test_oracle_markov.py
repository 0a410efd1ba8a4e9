"""The discrete-time diffusion oracle (Sec. "Simulating discrete-time diffusion",
eq. let_there_be_markov with D = diag(w)) against closed forms and invariants.

Pins: on a cycle C_n (2-regular) phi is a function of A whose eigenvalues follow from
A's, 2 cos(2 pi k / n): for the BTDW resolvent phi(lambda) = (1 - mu^2 a^2) /
((1 - mu^2 a^2) + 2 a^2 mu - a lambda) (eq. deformed with D = 2 I), so P = phi / w has
eigenvalues phi(lambda_k) / phi(2); on K_n with the exponential at mu = 0 the chain's
eigenvalues are 1 and exp(-beta n).  Invariants: P 1 = 1, pi P = pi, mass conservation,
convergence to pi."""

import numpy as np
import pytest

import synth
from oracle import genfun, laplacian, walks


def cycle(n):
    rp, ci = synth.cycle_graph(n)
    return walks.adjacency(n, rp, ci)


@pytest.mark.parametrize("n", [9, 12])
@pytest.mark.parametrize("mu", [0.0, 0.5, 1.0])
def test_cycle_resolvent_gap_closed_form(n, mu):
    A = cycle(n)
    a = 0.3  # below 1 / rho(Z_mu) = 1 / (2 - mu)
    ph = genfun.phi(A, mu, "res", a)
    f = lambda lam: (1 - mu * mu * a * a) / ((1 - mu * mu * a * a) + 2 * a * a * mu - a * lam)
    lam_P = np.sort([f(2 * np.cos(2 * np.pi * k / n)) / f(2.0) for k in range(n)])
    np.testing.assert_allclose(laplacian.markov_spectrum(ph), lam_P, rtol=0, atol=1e-13)
    l2, lmin, gap = laplacian.spectral_gap(ph)
    assert abs(l2 - lam_P[-2]) < 1e-13 and abs(lmin - lam_P[0]) < 1e-13
    assert abs(gap - (1 - max(abs(lam_P[-2]), abs(lam_P[0])))) < 1e-13


def test_complete_graph_exponential_gap():
    n, beta = 7, 0.4
    A = np.ones((n, n)) - np.eye(n)
    ph = genfun.phi(A, 0.0, "exp", beta)
    lam = laplacian.markov_spectrum(ph)
    assert abs(lam[-1] - 1.0) < 1e-13
    np.testing.assert_allclose(lam[:-1], np.exp(-beta * n), rtol=1e-11)
    assert abs(laplacian.spectral_gap(ph)[2] - (1 - np.exp(-beta * n))) < 1e-12


@pytest.mark.parametrize("kind,mu", [("res", 0.5), ("exp", 0.0), ("exp", 1.0)])
def test_chain_invariants(kind, mu):
    n = 60
    rp, ci = synth.erdos_renyi_gnm(n, 240, 5)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu)) if kind == "res" else 1.0 / lam
    ph = genfun.phi(A, mu, kind, param)
    P = laplacian.markov_transition(ph)
    pi = laplacian.stationary_distribution(ph)
    np.testing.assert_allclose(P.sum(1), 1.0, atol=1e-13)
    np.testing.assert_allclose(pi @ P, pi, atol=1e-15)
    rng = np.random.default_rng(1)
    P0 = rng.random((n, 3))
    P0 /= P0.sum(0)
    X = laplacian.markov_steps(ph, P0, 7)
    np.testing.assert_allclose(X.sum(0), 1.0, atol=1e-13)
    np.testing.assert_allclose(X, np.linalg.matrix_power(P.T, 7) @ P0, atol=1e-14)
    # the largest eigenvalue of P is 1 and the spectrum agrees with P's own eigenvalues
    ev = np.sort(np.linalg.eigvals(P).real)
    np.testing.assert_allclose(laplacian.markov_spectrum(ph), ev, atol=1e-10)
    if kind == "res":  # phi > 0 entrywise on a connected graph: the chain forgets p_0
        Xl = laplacian.markov_steps(ph, P0, 400)
        np.testing.assert_allclose(Xl, np.repeat(pi[:, None], 3, 1), atol=1e-8)
