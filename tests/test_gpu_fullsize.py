"""Parity at full size, in the launch configurations the benchmark times.

Barabasi-Albert n = 10^6, m = 5 (the benchmark graph, 1e7 nonzeros), FP32 blocks of 16
Rademacher columns with Krylov dimension 30, against the sparse FP64 oracle (truncated
series and CG on A_mu(alpha)) on the columns it can afford; the road-network stand-in
(n = 1.96e6) for the rational Krylov estimate, by properties that hold at any size
(its oracle is dense).
Tolerances as for the FP32 path elsewhere: phi X 2e-5, w 1e-5 relative."""

import numpy as np
import pytest

import synth
from oracle import sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


@pytest.fixture(scope="module")
def ba1m():
    n = 1_000_000
    rp, ci = synth.barabasi_albert(n, 5, seed=2026)
    return n, rp, ci, sparse.adjacency(n, rp, ci)


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def node_rel(a, b, mag):
    """Largest error of any node against that node's magnitude (phi >= 0 entrywise, so
    for Rademacher columns |(phi X)_ij| <= (phi 1)_i = w_i)."""
    return float(np.max(np.abs(a - b) / np.asarray(mag)[:, None]))


@pytest.mark.parametrize("mu", [0.0, 0.5, 1.0])
def test_series_block16_full_size(ctx, lib, ba1m, mu):
    n, rp, ci, As = ba1m
    print(f"[gpu] full size BA 1e6 exp mu={mu}", flush=True)
    g = lib.Graph(ctx, rp, ci)
    g.autotune(torch.float32, 16)
    lam = g.lambda_max()
    op = lib.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=30)
    X = synth.rademacher_block(n, 16, 3)
    PX = host(op.apply_phi(dev(X, torch.float32)))
    coeffs = np.array([lam ** -k / np.prod(np.arange(1, k + 1, dtype=np.float64)) for k in range(31)])
    cols = [0, 7, 15]
    ref = sparse.series_apply(As, mu, coeffs, X[:, cols])
    assert rel(PX[:, cols], ref) < 2e-5
    w = host(op.fdeg())
    wr = sparse.series_apply(As, mu, coeffs, np.ones((n, 1)))[:, 0]
    ew, ep = float(np.max(np.abs(w - wr) / wr)), node_rel(PX[:, cols], ref, wr)
    print(f"[gpu] per-node errors: w {ew:.1e}, phi X {ep:.1e}", flush=True)
    assert ew < 2e-5 and ep < 1e-4
    # L 1 = 0 at full size
    ones = torch.ones((n, 1), dtype=torch.float32, device="cuda")
    L1 = host(op.apply_L(ones))
    assert np.abs(L1).max() < 1e-5 * np.abs(w).max()


def test_resolvent_lanczos_block16_full_size(ctx, lib, ba1m):
    n, rp, ci, As = ba1m
    print("[gpu] full size BA 1e6 res mu=0.5 Lanczos", flush=True)
    g = lib.Graph(ctx, rp, ci)
    g.autotune(torch.float32, 16)
    rho = g.spectral_radius(0.5)
    alpha = 0.5 / rho
    op = lib.Operator(g, 0.5, "res", alpha, dtype=torch.float32, krylov_dim=30, rho_hint=rho)
    X = synth.rademacher_block(n, 16, 3)
    PX = host(op.apply_phi(dev(X, torch.float32)))
    cols = [2, 11]
    ref = sparse.phi_res_apply(As, 0.5, alpha, X[:, cols], rtol=1e-12)
    assert rel(PX[:, cols], ref) < 2e-5
    w = host(op.fdeg())
    wr = sparse.phi_res_apply(As, 0.5, alpha, np.ones((n, 1)), rtol=1e-12)[:, 0]
    ew, ep = float(np.max(np.abs(w - wr) / wr)), node_rel(PX[:, cols], ref, wr)
    print(f"[gpu] per-node errors: w {ew:.1e}, phi X {ep:.1e}", flush=True)
    assert ew < 2e-5 and ep < 1e-4


def test_resolvent_groups_reorth0_full_size(ctx, lib, ba1m):
    """The default workload's grouped Lanczos at full size: two resolvent operators side
    by side (32-wide lock-step processes with deferred normalisation, reorth 0: each
    new block projected against the current one only), and one operator's block beside
    the walk-degree processes of three operators (apply_fdeg with nx = 1), K = 30."""
    n, rp, ci, As = ba1m
    print("[gpu] full size BA 1e6 grouped resolvents reorth 0", flush=True)
    g = lib.Graph(ctx, rp, ci)
    for w_ in (32, 16):
        g.autotune(torch.float32, w_)
    mus = [0.5, 1.0, 0.25]
    rhos = [g.spectral_radius(mu) for mu in mus]
    ops = [lib.Operator(g, mu, "res", 0.5 / rho, dtype=torch.float32, krylov_dim=30, rho_hint=rho, reorth=0)
           for mu, rho in zip(mus, rhos)]
    X = synth.rademacher_block(n, 16, 3)
    Xd = dev(X, torch.float32)
    PX = host(lib.Multi(ops[:2]).apply_phi(Xd))
    Y, W = lib.Multi([ops[2], ops[0], ops[1]]).apply_fdeg(Xd, laplacian=False, nx=1)
    Y, W = host(Y), host(W)
    cols = [4, 13]
    for i, (mu, rho) in enumerate(zip(mus, rhos)):
        alpha = 0.5 / rho
        wr = sparse.phi_res_apply(As, mu, alpha, np.ones((n, 1)), rtol=1e-12)[:, 0]
        w = W[:, (i + 1) % 3]  # W's columns follow the second Multi's operator order
        ew = float(np.max(np.abs(w - wr) / wr))
        got = PX[:, [16 * i + c for c in cols]] if i < 2 else Y[:, cols]
        ref = sparse.phi_res_apply(As, mu, alpha, X[:, cols], rtol=1e-12)
        ep = node_rel(got, ref, wr)
        print(f"[gpu] mu={mu}: phi X {rel(got, ref):.1e} (per node {ep:.1e}), w per node {ew:.1e}", flush=True)
        assert rel(got, ref) < 2e-5 and ep < 1e-4 and ew < 2e-5


def test_markov_chain_full_size(ctx, lib, ba1m):
    n, rp, ci, As = ba1m
    print("[gpu] full size BA 1e6 markov chain", flush=True)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    op = lib.Operator(g, 1.0, "exp", 1.0 / lam, dtype=torch.float32, tol=1e-9)
    K = op.info()[0]
    starts = np.random.default_rng(590).choice(n, size=4, replace=False)
    P0 = synth.spike_block(n, starts)
    P1 = host(op.markov_step(dev(P0, torch.float32), steps=1))
    coeffs = np.array([lam ** -k / np.prod(np.arange(1, k + 1, dtype=np.float64)) for k in range(K + 1)])
    w = sparse.series_apply(As, 1.0, coeffs, np.ones((n, 1)))
    ref = sparse.series_apply(As, 1.0, coeffs, P0 / w)
    assert rel(P1, ref) < 2e-5
    P20 = host(op.markov_step(dev(P0, torch.float32), steps=20))
    np.testing.assert_allclose(P20.sum(0), 1.0, atol=1e-5)
    pi = host(op.markov_stationary())
    assert rel(pi, w[:, 0] / w.sum()) < 1e-5


def test_arnoldi_full_size(ctx, lib, ba1m):
    n, rp, ci, As = ba1m
    print("[gpu] full size BA 1e6 Arnoldi on the linearisation", flush=True)
    g = lib.Graph(ctx, rp, ci)
    mu = 0.5
    rhoZ = g.spectral_radius(mu)
    beta = 20.0 / rhoZ
    op = lib.Operator(g, mu, "exp", beta, dtype=torch.float32, krylov_dim=20, method="arnoldi")
    X = synth.rademacher_block(n, 16, 3)
    PX = host(op.apply_phi(dev(X, torch.float32)))
    cols = [1, 9]
    ref = sparse.phi_exp_apply(As, mu, beta, X[:, cols], tol=1e-12)
    assert rel(PX[:, cols], ref) < 2e-5


def test_return_probability_road_full_size(ctx, lib):
    """At t = 0, Y(0) = Omega / n exactly: p_hat(0) estimates tr(I) / n = 1 within its
    statistical error; p_hat stays in (0, 1] and decreases from there, with error
    estimates below p_hat."""
    print("[gpu] full size road stand-in return probability", flush=True)
    rp, ci = synth.road_grid(1400, 1400, 0.7, seed=7)
    n = len(rp) - 1
    g = lib.Graph(ctx, rp, ci)
    rhoZ = g.spectral_radius(1.0)
    op = lib.Operator(g, 1.0, "res", 1.0 / (1.0 + rhoZ), dtype=torch.float32, tol=1e-7, rho_hint=rhoZ)
    Om = lib.probes(ctx, n, 30, seed=2026, law="gauss", dtype=torch.float32)
    ts = np.linspace(0.0, 100.0, 12)
    p, e, poles, info = op.return_prob(Om, ts, 100.0, solve_tol=1e-6, max_iters=1000)
    assert abs(p[0] - 1.0) < 5 * e[0] + 1e-3
    assert np.all(p > 0) and np.all(p <= 1.0 + 1e-3) and p[-1] < 0.1 * p[0]
    assert np.all(e < p)
    assert info["solve_res"] <= 1e-6 and info["npoles"] >= 8
