"""Discrete-time diffusion (Sec. "Simulating discrete-time diffusion",
eq. let_there_be_markov with D = diag(w)) through the C ABI against the oracle.

Tolerances: chain steps and stationary distribution as the phi products they are made
of (FP64 1e-8, FP32 2e-5 relative).  Eigenvalue estimates: Lanczos Ritz values for the
extreme eigenvalues after 80 (FP64) / 60 (FP32) fully reorthogonalised steps, checked
to 1e-7 (FP64) and 1e-4 (FP32) absolute against the dense spectrum."""

import numpy as np
import pytest

import synth
from oracle import genfun, laplacian, sparse, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def distributions(n, b, seed):
    rng = np.random.default_rng(seed)
    P0 = rng.random((n, b))
    P0[:, 0] = 0.0
    P0[3, 0] = 1.0  # a point mass
    return P0 / P0.sum(0)


def er_graph():
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 2400, 13)
    return n, rp, ci, walks.adjacency(n, rp, ci)


@pytest.mark.parametrize("mu,kind,method", [(0.0, "res", "lanczos"), (0.5, "res", "lanczos"),
                                            (1.0, "res", "recurrence"), (0.0, "exp", "lanczos"),
                                            (0.5, "exp", "recurrence")])
def test_markov_fp64_matches_dense(ctx, lib, mu, kind, method):
    print(f"[gpu] markov fp64 mu={mu} {kind} {method}", flush=True)
    n, rp, ci, A = er_graph()
    g = lib.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu)) if kind == "res" else 1.0 / lam
    # the resolvent series at alpha rho(Z_mu) = 1/2 needs about 45 terms for 1e-13
    K = 40 if method == "lanczos" else (45 if kind == "res" else 0)
    op = lib.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=K, method=method, tol=1e-14)
    ph = genfun.phi(A, mu, kind, param)
    P0 = distributions(n, 4, 1)
    X3 = host(op.markov_step(dev(P0, torch.float64), steps=3))
    ref = laplacian.markov_steps(ph, P0, 3)
    assert np.linalg.norm(X3 - ref) < 1e-8 * np.linalg.norm(ref)
    np.testing.assert_allclose(X3.sum(0), 1.0, atol=1e-10)
    X1 = op.markov_step(dev(P0, torch.float64), steps=1)
    X2 = host(op.markov_step(op.markov_step(X1, steps=1), steps=1))
    assert np.linalg.norm(X2 - X3) < 1e-12 * np.linalg.norm(ref)
    pi = host(op.markov_stationary())
    pr = laplacian.stationary_distribution(ph)
    assert np.linalg.norm(pi - pr) < 1e-10 * np.linalg.norm(pr)
    l2, lmin, gap = op.markov_gap(outer_dim=80)
    r2, rmin, rgap = laplacian.spectral_gap(ph)
    assert abs(l2 - r2) < 1e-7 and abs(lmin - rmin) < 1e-7 and abs(gap - rgap) < 1e-7, (l2, r2, lmin, rmin)


def test_markov_fp32_ba_resolvent(ctx, lib):
    print("[gpu] markov fp32 BA", flush=True)
    n = 3000
    rp, ci = synth.barabasi_albert(n, 4, 29)
    As = sparse.adjacency(n, rp, ci)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    mu = 0.5
    alpha = 0.5 / g.spectral_radius(mu)
    op = lib.Operator(g, mu, "res", alpha, dtype=torch.float32, krylov_dim=30)
    P0 = distributions(n, 16, 2)
    X = host(op.markov_step(dev(P0, torch.float32), steps=2))
    w = sparse.fdeg(As, mu, "res", alpha)
    ref = P0
    for _ in range(2):
        ref = sparse.phi_apply(As, mu, "res", alpha, ref / w[:, None])
    assert np.linalg.norm(X - ref) < 2e-5 * np.linalg.norm(ref)
    ph = genfun.phi(A, mu, "res", alpha)
    l2, lmin, gap = op.markov_gap(outer_dim=60)
    r2, rmin, rgap = laplacian.spectral_gap(ph)
    assert abs(l2 - r2) < 1e-4 and abs(lmin - rmin) < 1e-4 and abs(gap - rgap) < 1e-4, (l2, r2, lmin, rmin)


def test_markov_fig1_stationary(ctx, lib):
    """The stationary distributions printed in Fig. 1 from the GPU chain."""
    from test_oracle_genfun import load_fig1
    rp, ci = synth.toy_g58()
    g = lib.Graph(ctx, rp, ci)
    lam = 3.1964027540390294
    gold = load_fig1()
    for key, (mu, kind, param) in {"res": (0.0, "res", 1 / (2 * lam)), "exp": (0.0, "exp", 1.0)}.items():
        pi = host(lib.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=30).markov_stationary())
        for node, val in gold[key].items():
            assert abs(pi[node - 1] - val) < 1e-13


def test_markov_rejects_bad_arguments(ctx, lib):
    n, rp, ci, A = er_graph()
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.0, "res", 0.5 / np.linalg.eigvalsh(A)[-1], dtype=torch.float64, krylov_dim=20)
    X = dev(distributions(n, 2, 3), torch.float64)
    with pytest.raises(lib.WLError, match="EINVAL"):
        op.markov_step(X, steps=0)
    with pytest.raises(lib.WLError, match="EINVAL"):
        op.markov_gap(outer_dim=1)


def test_markov_edgeless_graph(ctx, lib):
    """No edges: phi = I, P = I: distributions stay put, pi is uniform, and every
    eigenvalue of P is 1 (gap 0)."""
    print("[gpu] markov edgeless graph", flush=True)
    n = 30
    g = lib.Graph(ctx, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), validate=True)
    op = lib.Operator(g, 0.5, "exp", 0.4, dtype=torch.float64, krylov_dim=5)
    P0 = distributions(n, 3, 4)
    np.testing.assert_allclose(host(op.markov_step(dev(P0, torch.float64), steps=5)), P0, atol=1e-14)
    np.testing.assert_allclose(host(op.markov_stationary()), np.full(n, 1.0 / n), atol=1e-15)
    l2, lmin, gap = op.markov_gap(outer_dim=10)
    assert abs(l2 - 1.0) < 1e-12 and abs(lmin - 1.0) < 1e-12 and abs(gap) < 1e-12
