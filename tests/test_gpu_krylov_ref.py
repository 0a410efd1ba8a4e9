"""FP32 Krylov path against the same-K FP64 Krylov reference (oracle.krylov) on an
R-MAT graph beyond dense sizes, in the configuration of the large diffusion workload:
R-MAT scale 16 (edge factor 16, a = .57, b = c = .19; hub rows of degree ~10^4 take
the whole-workgroup path), walk Laplacian of mu = 0.5 with exponential weights
(beta = 1 / lambda_max, inner series degree from the tail bound at 1e-9), 32 sparse
probability vectors (16 random non-isolated nodes each), 40 outer block Lanczos steps,
t in {0.1, 1, 10}.  The same K, the same start block and the same inner degree on both
sides: the difference is the kernels' FP32 rounding (contract 1e-4); the method's own
truncation error is reported beside it (the reference's a-posteriori estimate)."""

import numpy as np
import pytest

import synth
from oracle import krylov, sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rmat16():
    rp, ci = synth.rmat(16, 16, 0.57, 0.19, 0.19, 1616)
    n = len(rp) - 1
    return n, rp, ci, sparse.adjacency(n, rp, ci)


def sparse_starts(rp, b, seed):
    n = len(rp) - 1
    deg = np.diff(rp)
    pool = np.nonzero(deg > 0)[0]
    rng = np.random.default_rng(seed)
    U0 = np.zeros((n, b))
    for j in range(b):
        U0[rng.choice(pool, size=16, replace=False), j] = 1.0 / 16
    return U0


def test_diffusion_same_k_reference(lib, rmat16):
    n, rp, ci, As = rmat16
    print(f"[gpu] same-K diffusion R-MAT 16 n={n} nnz={len(ci)} max degree {np.diff(rp).max()}", flush=True)
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci, validate=True)
    lam = g.lambda_max()
    mu, b, K, ts = 0.5, 32, 40, [0.1, 1.0, 10.0]
    op = lib.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, tol=1e-9)
    Kin = op.info()[0]
    U0 = sparse_starts(rp, b, 25)
    outs, gerr = op.expv(torch.tensor(U0, dtype=torch.float32, device="cuda"), ts, outer_dim=K)
    c = krylov.exp_coefficients(1.0 / lam, Kin)
    w = krylov.series_apply(As, mu, c, np.ones((n, 1)))[:, 0]
    refs, rerr = krylov.expv_lanczos(lambda X: krylov.series_apply(As, mu, c, X), w, U0, ts, K, reorth="full")
    for t, o, r, ge, re in zip(ts, outs, refs, gerr, rerr):
        y = o.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(y - r) / np.linalg.norm(r)
        node = float(np.max(np.abs(y - r)) / np.max(np.abs(r)))
        print(f"[gpu] t={t}: FP32 vs same-K FP64 {err:.2e} (max node {node:.2e}); method error estimate "
              f"{re:.2e} (library's {ge:.2e}); inner degree {Kin}", flush=True)
        assert err < 1e-4 and node < 1e-4, (t, err, node)
        # mass is conserved: 1^T exp(-t L) = 1^T since L 1 = 0
        np.testing.assert_allclose(y.sum(0), U0.sum(0), rtol=1e-5)
        # the library's a-posteriori estimate has the order of the reference's
        assert ge < 10 * re + 1e-6 and re < 10 * ge + 1e-6, (t, ge, re)


def test_resolvent_lanczos_same_k_reference(lib, rmat16):
    """Block Lanczos on A_mu(alpha), 16 Rademacher columns, K = 30, local
    reorthogonalisation on both sides: FP32 against the FP64 same-K reference, and the
    method error (same-K reference against the converged solve) reported beside it."""
    n, rp, ci, As = rmat16
    print("[gpu] same-K resolvent Lanczos R-MAT 16", flush=True)
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci)
    mu = 0.5
    rho = g.spectral_radius(mu)
    alpha = 0.5 / rho
    op = lib.Operator(g, mu, "res", alpha, dtype=torch.float32, krylov_dim=30, rho_hint=rho)
    X = synth.rademacher_block(n, 16, 3)
    PX = op.apply_phi(torch.tensor(X, dtype=torch.float32, device="cuda")).cpu().numpy().astype(np.float64)
    ref = krylov.phi_resolvent_lanczos(As, mu, alpha, X, 30, reorth="local")
    exact = sparse.phi_res_apply(As, mu, alpha, X[:, :2], rtol=1e-13)
    w = sparse.phi_res_apply(As, mu, alpha, np.ones((n, 1)), rtol=1e-13)[:, 0]
    err = np.linalg.norm(PX - ref) / np.linalg.norm(ref)
    node = float(np.max(np.abs(PX - ref) / w[:, None]))
    meth = np.linalg.norm(ref[:, :2] - exact) / np.linalg.norm(exact)
    print(f"[gpu] resolvent: FP32 vs same-K FP64 {err:.2e} (max node / w {node:.2e}); method error {meth:.2e}",
          flush=True)
    assert err < 2e-5 and node < 1e-4


@pytest.mark.parametrize("K", [8, 16, 30])
def test_rank_deficient_block_same_k(lib, K):
    """A start block of rank 4 in 16 columns (12 zero columns) on a small graph with
    many components (a 9 x 11 lattice with edges kept w.p. 0.35: isolated nodes and
    small pieces, n = 99): the block Krylov space grows by 4 per step, so K steps are
    K steps here too (the step count is capped by n + 1, not by n / b + 1, which would
    stop at 8 and leave a 1e-2 error at any requested K).  phi X of the resolvent
    (mu = 1) in FP64 against the oracle's same-K block Lanczos on the rank-4 block."""
    print(f"[gpu] rank-deficient start block, same-K reference K={K}", flush=True)
    rp, ci = synth.road_grid(9, 11, 0.35, seed=11)
    n = len(rp) - 1
    As = sparse.adjacency(n, rp, ci)
    from oracle import genfun, walks
    Ad = walks.adjacency(n, rp, ci)
    alpha = 0.5 / walks.spectral_radius(walks.linearisation(Ad, 1.0))
    X = synth.gaussian_block(n, 16, seed=5)
    X[:, 4:] = 0.0
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float64, krylov_dim=K, method="lanczos", tol=1e-14)
    Y = op.apply_phi(torch.tensor(X, dtype=torch.float64, device="cuda")).cpu().numpy()
    ref = krylov.phi_resolvent_lanczos(As, 1.0, alpha, X[:, :4].copy(), K)
    exact = genfun.phi(Ad, 1.0, "res", alpha) @ X[:, :4]
    scale = np.abs(exact).max()
    err_ref = np.abs(Y[:, :4] - ref).max() / scale
    err_exact = np.abs(Y[:, :4] - exact).max() / scale
    print(f"[gpu]   vs same-K {err_ref:.2e}, vs exact {err_exact:.2e}", flush=True)
    assert err_ref < 1e-10, err_ref
    assert np.abs(Y[:, 4:]).max() == 0.0
    if K == 30:
        assert err_exact < 1e-12, err_exact


def test_rank_deficient_diffusion_outer_steps(lib):
    """exp(-t L) U0 with U0 of rank 2 in 8 columns on the same 99-node lattice: the outer
    Lanczos space grows by 2 per step, so 60 steps (120 > n) reach an invariant space and
    the result is exact to rounding.  (Its former cap of ceil(n / b) = 13 steps held it
    to 26 dimensions.)  FP64, against the dense exponential of the dense walk Laplacian."""
    print("[gpu] rank-2 diffusion start block, outer steps", flush=True)
    from oracle import genfun, laplacian, walks
    import scipy.linalg as sla
    rp, ci = synth.road_grid(9, 11, 0.35, seed=11)
    n = len(rp) - 1
    Ad = walks.adjacency(n, rp, ci)
    beta = 1.0 / np.linalg.eigvalsh(Ad)[-1]
    L = laplacian.walk_laplacian(genfun.phi(Ad, 0.5, "exp", beta))
    G = synth.gaussian_block(n, 2, seed=7)
    U0 = np.concatenate([G, G @ np.array([[1.0, 2.0, 0.5, 0.0, 1.0, -1.0], [1.0, -1.0, 3.0, 0.0, 0.0, 2.0]])], axis=1)
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.5, "exp", beta, dtype=torch.float64, tol=1e-14)
    ts = [0.5, 5.0]
    outs, _ = op.expv(torch.tensor(U0, dtype=torch.float64, device="cuda"), ts, outer_dim=60)
    for t, y in zip(ts, outs):
        ref = sla.expm(-t * L) @ U0
        err = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
        print(f"[gpu]   t={t}: relative error {err:.2e}", flush=True)
        assert err < 1e-9, (t, err)
