"""Exponential weights by block Arnoldi on the linearisation Z (eq. Zdef, Prop.
"whe-we-converge": phi X = X + [I O] beta phi_1(beta Z) [q_1 X; q_2 X]) through the C
ABI against the oracle's dense linearisation (phi_1 of the 2n x 2n matrix by expm of the
augmented matrix) and its sparse truncated series.

Tolerances, relative Frobenius: FP64 1e-9 once the Krylov space has converged (40 block
steps at beta rho(Z) = 20), 1e-11 when it spans all of R^{2n}; FP32 1e-4."""

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


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("mu", [0.0, 0.5, 1.0])
def test_fp64_matches_dense_linearisation(ctx, lib, mu):
    print(f"[gpu] arnoldi fp64 mu={mu}", flush=True)
    n = 300
    rp, ci = synth.barabasi_albert(n, 3, 41)
    A = walks.adjacency(n, rp, ci)
    beta = 20.0 / walks.spectral_radius(walks.linearisation(A, mu))
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, "exp", beta, dtype=torch.float64, krylov_dim=40, method="arnoldi")
    assert op.info() == (40, lib.WL_M_ARNOLDI)
    ph = genfun.phi(A, mu, "exp", beta)
    X = synth.gaussian_block(n, 4, seed=2)
    Y = host(op.apply_phi(dev(X, torch.float64)))
    assert rel(Y, ph @ X) < 1e-9
    w = host(op.fdeg())
    assert rel(w, ph.sum(1)) < 1e-9
    LX = host(op.apply_L(dev(X, torch.float64)))
    ref = laplacian.apply_laplacian(ph, X)
    assert rel(LX, ref) < 1e-9


def test_error_decreases_with_steps(ctx, lib):
    print("[gpu] arnoldi convergence in the number of steps", flush=True)
    n = 300
    rp, ci = synth.barabasi_albert(n, 3, 7)
    A = walks.adjacency(n, rp, ci)
    mu = 0.5
    beta = 30.0 / walks.spectral_radius(walks.linearisation(A, mu))
    g = lib.Graph(ctx, rp, ci)
    ph = genfun.phi(A, mu, "exp", beta)
    X = synth.gaussian_block(n, 2, seed=5)
    errs = []
    for K in (6, 12, 24, 48):
        op = lib.Operator(g, mu, "exp", beta, dtype=torch.float64, krylov_dim=K, method="arnoldi")
        errs.append(rel(host(op.apply_phi(dev(X, torch.float64))), ph @ X))
    # decreasing until the rounding floor of the comparison (~1e-12) is reached
    assert all(e2 < e1 or e2 < 1e-10 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[0] > 1e-4 and errs[-1] < 1e-10, errs


def test_full_space_is_exact(ctx, lib):
    print("[gpu] arnoldi exhausting the space", flush=True)
    rp, ci = synth.toy_g58()
    n = len(rp) - 1
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "exp", 0.8, dtype=torch.float64, krylov_dim=50, method="arnoldi")
    X = synth.gaussian_block(n, 2, seed=1)
    Y = host(op.apply_phi(dev(X, torch.float64)))
    assert rel(Y, genfun.phi(A, 1.0, "exp", 0.8) @ X) < 1e-11


def test_rank_deficient_block_reaches_full_space(ctx, lib):
    """A start block of rank 2 in 6 columns on a 40-node graph with several components: the
    space of Z grows by 2 per step, so the step count may not stop at 2n / b (13 here);
    with 50 steps it reaches an invariant space and phi X is exact to rounding."""
    print("[gpu] arnoldi rank-deficient start block", flush=True)
    rp, ci = synth.road_grid(5, 8, 0.5, seed=3)
    n = len(rp) - 1
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.5, "exp", 0.8, dtype=torch.float64, krylov_dim=50, method="arnoldi")
    G = synth.gaussian_block(n, 2, seed=4)
    X = np.concatenate([G, G @ np.array([[1.0, 0.5, -2.0, 0.0], [1.0, 3.0, 1.0, 0.0]])], axis=1)
    Y = host(op.apply_phi(dev(X, torch.float64)))
    assert rel(Y, genfun.phi(A, 0.5, "exp", 0.8) @ X) < 1e-11


def test_fp32_ba_against_sparse_series(ctx, lib):
    print("[gpu] arnoldi fp32 BA n=4000 b=16", flush=True)
    n = 4000
    rp, ci = synth.barabasi_albert(n, 4, 13)
    As = sparse.adjacency(n, rp, ci)
    mu = 0.5
    beta = 25.0 / sparse.rho_Z(As, mu)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, "exp", beta, dtype=torch.float32, krylov_dim=40, method="arnoldi")
    X = synth.gaussian_block(n, 16, seed=3)
    Y = host(op.apply_phi(dev(X, torch.float32)))
    ref = sparse.phi_exp_apply(As, mu, beta, X, tol=1e-14)
    assert rel(Y, ref) < 1e-4


def test_rejected_uses(ctx, lib):
    print("[gpu] arnoldi rejected uses", flush=True)
    rp, ci = synth.barabasi_albert(100, 2, 1)
    g = lib.Graph(ctx, rp, ci)
    with pytest.raises(lib.WLError):
        lib.Operator(g, 0.5, "res", 0.1, dtype=torch.float64, krylov_dim=10, method="arnoldi")
    with pytest.raises(lib.WLError):
        lib.Operator(g, 0.5, "exp", 0.1, dtype=torch.float64, method="arnoldi")
    op = lib.Operator(g, 0.5, "exp", 0.1, dtype=torch.float64, krylov_dim=10, method="arnoldi")
    with pytest.raises(lib.WLError):
        lib.Multi([op, op])


def test_fp32_series_large_beta(ctx, lib):
    """The truncated series at beta lambda_max ~ 30 (regression: with the iterates scaled
    by beta they grew like (beta lambda_max)^k and overflowed FP32), alone and side by
    side with a second operator."""
    print("[gpu] series fp32 at large beta", flush=True)
    n = 4000
    rp, ci = synth.barabasi_albert(n, 4, 13)
    As = sparse.adjacency(n, rp, ci)
    mu = 0.5
    beta = 25.0 / sparse.rho_Z(As, mu)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, "exp", beta, dtype=torch.float32, tol=1e-8)
    assert op.info()[0] > 40
    X = synth.gaussian_block(n, 16, seed=3)
    ref = sparse.phi_exp_apply(As, mu, beta, X, tol=1e-14)
    Y = host(op.apply_phi(dev(X, torch.float32)))
    assert np.all(np.isfinite(Y)) and rel(Y, ref) < 1e-4
    other = lib.Operator(g, mu, "exp", 0.5 * beta, dtype=torch.float32, tol=1e-8)
    Ym = host(lib.Multi([op, other]).apply_phi(dev(X, torch.float32)))
    assert rel(Ym[:, :16], ref) < 1e-4
    assert rel(Ym[:, 16:], sparse.phi_exp_apply(As, mu, 0.5 * beta, X, tol=1e-14)) < 1e-4


def test_edgeless_graph(ctx, lib):
    """No edges: A = D = 0, the start block [q_1 X; q_2 X] vanishes and phi = c_0 I."""
    print("[gpu] arnoldi edgeless graph", flush=True)
    n = 20
    g = lib.Graph(ctx, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), validate=True)
    op = lib.Operator(g, 0.5, "exp", 0.7, dtype=torch.float64, krylov_dim=4, method="arnoldi")
    X = synth.gaussian_block(n, 3, seed=2)
    np.testing.assert_allclose(host(op.apply_phi(dev(X, torch.float64))), X, atol=1e-15)
