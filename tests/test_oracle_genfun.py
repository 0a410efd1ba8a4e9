"""Pins of the oracle's generating functions and Laplacians (Sec. 3 and 4):
agreement of independent routes, library special cases, closed forms on
regular graphs, the paper's structural propositions and its Fig. 1."""

import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import genfun, laplacian, walks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def irregular():
    rp, ci = synth.erdos_renyi_gnm(40, 90, seed=11)
    return walks.adjacency(40, rp, ci)


@pytest.mark.parametrize("mu", [0.0, 0.25, 0.5, 0.75, 1.0])
def test_resolvent_three_routes(mu):
    A = irregular()
    rho = walks.spectral_radius(walks.linearisation(A, mu))
    alpha = 0.5 / rho
    closed = genfun.phi_resolvent_closed(A, mu, alpha)
    lin = genfun.phi_resolvent_linearised(A, mu, alpha)
    series = genfun.phi_series(A, mu, genfun.coefficients("res", alpha, 80))
    np.testing.assert_allclose(closed, lin, rtol=0, atol=1e-13 * np.abs(closed).max())
    np.testing.assert_allclose(closed, series, rtol=0, atol=1e-12 * np.abs(closed).max())


@pytest.mark.parametrize("mu", [0.0, 0.25, 0.5, 0.75, 1.0])
def test_exponential_two_routes(mu):
    A = irregular()
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    lin = genfun.phi_exponential_linearised(A, mu, beta)
    series = genfun.phi_series(A, mu, genfun.coefficients("exp", beta, 40))
    np.testing.assert_allclose(lin, series, rtol=0, atol=1e-13 * np.abs(series).max())


def test_mu0_reduces_to_library_matrix_functions():
    A = irregular()
    lam = np.linalg.eigvalsh(A)[-1]
    np.testing.assert_allclose(genfun.phi(A, 0.0, "exp", 1.0 / lam), sla.expm(A / lam), atol=1e-13)
    np.testing.assert_allclose(genfun.phi(A, 0.0, "res", 0.5 / lam), sla.inv(np.eye(40) - 0.5 / lam * A), atol=1e-13)


def test_mu1_resolvent_is_eq_deformed():
    """phi (I - a A - a^2 (I - D)) = (1 - a^2) I  (eq. deformed)."""
    A = irregular()
    a = 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))
    D = np.diag(A.sum(1))
    ph = genfun.phi_series(A, 1.0, genfun.coefficients("res", a, 120))
    np.testing.assert_allclose(ph @ (np.eye(40) - a * A - a * a * (np.eye(40) - D)), (1 - a * a) * np.eye(40), atol=1e-12)


REGULAR = {
    "cycle12": (12, 2) + synth.cycle_graph(12),
    "circ20_4": (20, 4) + synth.circulant_graph(20, [1, 3]),
    "circ40_6": (40, 6) + synth.circulant_graph(40, [1, 2, 5]),
    "k6": (6, 5) + synth.complete_graph(6),
    "q4": (16, 4) + synth.hypercube_graph(4),
}


@pytest.mark.parametrize("name", list(REGULAR))
@pytest.mark.parametrize("mu", [0.0, 0.25, 0.5, 0.75, 1.0])
def test_regular_graph_closed_forms(name, mu):
    """d-regular: (q_k 1)_i = d (d - mu)^{k-1}, so
    w_res = (1 + mu a) / (1 - a (d - mu)),  w_exp = 1 + d (e^{b (d - mu)} - 1) / (d - mu),
    and rho(Z_mu) = d - mu."""
    n, d, rp, ci = REGULAR[name]
    A = walks.adjacency(n, rp, ci)
    rho = walks.spectral_radius(walks.linearisation(A, mu))
    assert abs(rho - (d - mu)) < 1e-8 * d
    a = 0.5 / (d - mu)
    w = laplacian.walk_degree(genfun.phi(A, mu, "res", a))
    np.testing.assert_allclose(w, (1 + mu * a) / (1 - a * (d - mu)), rtol=1e-13)
    b = 0.7 / d
    w = laplacian.walk_degree(genfun.phi(A, mu, "exp", b))
    np.testing.assert_allclose(w, 1 + d * math.expm1(b * (d - mu)) / (d - mu), rtol=1e-13)


def test_first_walk_coefficient_gives_standard_laplacian():
    """c = (0, 1, 0, ...) (Sec. 3.1) gives L = D - A, for every mu."""
    A = irregular()
    for mu in (0.0, 0.5, 1.0):
        ph = genfun.phi_series(A, mu, np.array([0.0, 1.0, 0.0, 0.0]))
        np.testing.assert_array_equal(laplacian.walk_laplacian(ph), np.diag(A.sum(1)) - A)


@pytest.mark.parametrize("mu", [0.0, 0.5, 1.0])
@pytest.mark.parametrize("kind", ["res", "exp"])
def test_laplacian_properties(mu, kind):
    """Prop. "still-an-mmatrix" / "still-again-an-mmatrix": symmetric, L 1 = 0,
    and a (singular) M-matrix since phi >= 0 entrywise for these weights."""
    A = irregular()
    param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu)) if kind == "res" else 1.0 / np.linalg.eigvalsh(A)[-1]
    ph = genfun.phi(A, mu, kind, param)
    assert ph.min() >= -1e-14
    L = laplacian.walk_laplacian(ph)
    np.testing.assert_allclose(L, L.T, atol=1e-13)
    np.testing.assert_allclose(L @ np.ones(40), 0, atol=1e-12)
    off = L - np.diag(np.diag(L))
    assert off.max() <= 1e-14
    assert np.linalg.eigvalsh(L).min() > -1e-11


def test_mu_continuity():
    A = irregular()
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    w = [laplacian.walk_degree(genfun.phi(A, mu, "exp", beta)) for mu in np.linspace(0, 1, 11)]
    for a, b in zip(w, w[1:]):
        assert np.all(b <= a + 1e-12)  # more downweighting, fewer weighted walks
        assert np.abs(a - b).max() < 0.2 * np.abs(a).max()


def test_exp_tail_bound_holds():
    A = irregular()
    lam = np.linalg.eigvalsh(A)[-1]
    beta = 1.0 / lam
    exact = genfun.phi(A, 0.5, "exp", beta)
    for K in (3, 6, 10):
        trunc = genfun.phi_series(A, 0.5, genfun.coefficients("exp", beta, K))
        assert np.linalg.norm(exact - trunc, 2) <= genfun.exp_tail_bound(beta, lam, K) * (1 + 1e-12)


def load_fig1():
    rows = {}
    with open(os.path.join(GOLDEN, "fig1_stationary.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, node, val = line.split()
            rows.setdefault(key, {})[int(node)] = float(val)
    return rows


def test_fig1_stationary_distributions():
    """Fig. 1 (Sec. 5.1): stationary distribution pi = w / sum(w) of
    P = diag(w)^{-1} phi on G_{5,8}; alpha = 1/(2 rho(A)) for the resolvent,
    beta = 1 for the exponential."""
    rp, ci = synth.toy_g58()
    A = walks.adjacency(13, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    assert abs(lam - 3.1964027540390294) < 1e-13
    gold = load_fig1()
    cases = {
        "L": A,
        "res": genfun.phi(A, 0.0, "res", 1.0 / (2 * lam)),
        "exp": genfun.phi(A, 0.0, "exp", 1.0),
        # printed NBT-exp bar: reproduced by the [O I] selector (see genfun)
        "nbtexp": genfun.phi_exponential_linearised(A, 1.0, 1.0, selector="O I"),
    }
    for key, ph in cases.items():
        pi = laplacian.stationary_distribution(ph)
        for node, val in gold[key].items():
            assert abs(pi[node - 1] - val) < 1e-14, (key, node, pi[node - 1], val)
        # the chain's stationary vector really is stationary
        P = laplacian.markov_transition(ph)
        np.testing.assert_allclose(pi @ P, pi, atol=1e-15)


def test_fig1_nbtexp_printed_bar_differs_from_displayed_formula():
    """Documents the inconsistency: eq. exp-based-laplacian ([I O] selector) does not
    give the printed bar; the exact rationals over 337 are the [O I] values."""
    rp, ci = synth.toy_g58()
    A = walks.adjacency(13, rp, ci)
    gold = load_fig1()["nbtexp"]
    pi_io = laplacian.stationary_distribution(genfun.phi_exponential_linearised(A, 1.0, 1.0))
    assert max(abs(pi_io[k - 1] - v) for k, v in gold.items()) > 0.1
    for k, v in gold.items():
        assert abs(v * 337 * 2 - round(v * 337 * 2)) < 1e-9
