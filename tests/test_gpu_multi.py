"""Several operators of one graph evaluated side by side (one sparse product per step
for all of them) against the single operators and the oracle.
Truncated series: FP64 1e-8 against the oracle, 1e-12 against the single operators
(only the summation order of the sparse products differs); FP32 2e-5 / 1e-6.
Lanczos groups (Sec. 4.1 run per group in lock step): FP64 1e-8 against the oracle and
1e-10 against the single operators (grouped kernels sum in another order, amplified by
the Krylov recurrence); FP32 2e-5 against the oracle (scaled as the single-operator
tests) and 2e-5 against the single operators."""

import numpy as np
import pytest

import synth
from oracle import genfun, laplacian, sparse, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def test_multi_fp64_matches_single_and_dense(ctx, lib):
    print("[gpu] multi fp64", flush=True)
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    specs = [(0.0, "exp", 1.0 / lam, 0), (0.5, "res", 0.5 / lam, 45), (1.0, "exp", 1.0 / lam, 0),
             (0.25, "exp", 0.5 / lam, 0)]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float64, krylov_dim=K, method="recurrence")
           for mu, f, p, K in specs]
    assert len({op.info()[0] for op in ops}) > 1  # different degrees in one pass
    multi = lib.Multi(ops)
    b = 3
    X = synth.gaussian_block(n, b, 5)
    Xd = dev(X, torch.float64)
    W = host(multi.fdeg())
    PX = host(multi.apply_phi(Xd))
    LX = host(multi.apply_L(Xd))
    for i, (op, (mu, f, p, K)) in enumerate(zip(ops, specs)):
        ph = genfun.phi(A, mu, f, p)
        w = ph.sum(1)
        cols = slice(i * b, (i + 1) * b)
        np.testing.assert_allclose(W[:, i], host(op.fdeg()), rtol=1e-12)
        assert np.linalg.norm(W[:, i] - w) < 1e-8 * np.linalg.norm(w)
        assert np.linalg.norm(PX[:, cols] - host(op.apply_phi(Xd))) < 1e-12 * np.linalg.norm(PX[:, cols])
        assert np.linalg.norm(PX[:, cols] - ph @ X) < 1e-8 * np.linalg.norm(ph @ X)
        scale = np.linalg.norm(w[:, None] * X) + np.linalg.norm(ph @ X)
        assert np.linalg.norm(LX[:, cols] - host(op.apply_L(Xd))) < 1e-12 * scale
        assert np.linalg.norm(LX[:, cols] - laplacian.apply_laplacian(ph, X)) < 1e-8 * scale


def test_multi_fp32_four_operators_block16(ctx, lib):
    """Four operators x 16 columns: rows of 64 FP32 values, two whole cache lines."""
    print("[gpu] multi fp32 BA20k", flush=True)
    n = 20000
    rp, ci = synth.barabasi_albert(n, 5, 11)
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    mus = [0.0, 0.25, 0.5, 1.0]
    ops = [lib.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=30) for mu in mus]
    multi = lib.Multi(ops)
    X = synth.rademacher_block(n, 16, 3)
    Xd = dev(X, torch.float32)
    LX = host(multi.apply_L(Xd))
    for i, (mu, op) in enumerate(zip(mus, ops)):
        cols = slice(16 * i, 16 * (i + 1))
        single = host(op.apply_L(Xd))
        wr = sparse.fdeg(As, mu, "exp", 1.0 / lam)
        pr = sparse.phi_apply(As, mu, "exp", 1.0 / lam, X)
        scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(pr)
        assert np.linalg.norm(LX[:, cols] - single) < 1e-6 * scale
        assert np.linalg.norm(LX[:, cols] - (wr[:, None] * X - pr)) < 2e-5 * scale


def test_multi_rejects_mixed_methods_and_graphs(ctx, lib):
    n = 300
    rp, ci = synth.erdos_renyi_gnm(n, 900, 2)
    g1, g2 = lib.Graph(ctx, rp, ci), lib.Graph(ctx, rp, ci)
    lam = g1.lambda_max()
    lan = lib.Operator(g1, 0.0, "res", 0.5 / lam, dtype=torch.float64, krylov_dim=20)  # Lanczos
    rec1 = lib.Operator(g1, 0.5, "exp", 1.0 / lam, dtype=torch.float64)
    rec2 = lib.Operator(g2, 0.5, "exp", 1.0 / lam, dtype=torch.float64)
    with pytest.raises(lib.WLError, match="UNSUPPORTED"):
        lib.Multi([rec1, lan])
    with pytest.raises(lib.WLError, match="EINVAL"):
        lib.Multi([rec1, rec2])


def _res_alpha(g, mu, lam):
    return 0.5 / (g.spectral_radius(mu) if mu > 0 else lam)


def test_multi_lanczos_fp64_single_columns_and_fallback(ctx, lib):
    """FP64 Lanczos groups: walk degrees through the grouped single-column kernels; a
    3-wide block is evaluated operator by operator (no grouped kernels for it)."""
    print("[gpu] multi lanczos fp64", flush=True)
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    specs = [(0.0, "res", 0.5 / lam), (0.5, "res", _res_alpha(g, 0.5, lam)), (1.0, "res", _res_alpha(g, 1.0, lam)),
             (0.0, "exp", 1.0 / lam)]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float64, krylov_dim=40, method="lanczos") for mu, f, p in specs]
    multi = lib.Multi(ops)
    W = host(multi.fdeg())
    b = 3
    X = synth.gaussian_block(n, b, 5)
    Xd = dev(X, torch.float64)
    LX = host(multi.apply_L(Xd))
    PX = host(multi.apply_phi(Xd))
    for i, (op, (mu, f, p)) in enumerate(zip(ops, specs)):
        ph = genfun.phi(A, mu, f, p)
        w = ph.sum(1)
        assert np.linalg.norm(W[:, i] - w) < 1e-8 * np.linalg.norm(w), (mu, f)
        assert np.linalg.norm(W[:, i] - host(op.fdeg())) < 1e-10 * np.linalg.norm(w), (mu, f)
        cols = slice(i * b, (i + 1) * b)
        assert np.linalg.norm(PX[:, cols] - ph @ X) < 1e-8 * np.linalg.norm(ph @ X), (mu, f)
        scale = np.linalg.norm(w[:, None] * X) + np.linalg.norm(ph @ X)
        assert np.linalg.norm(LX[:, cols] - laplacian.apply_laplacian(ph, X)) < 1e-8 * scale, (mu, f)
        np.testing.assert_allclose(PX[:, cols], host(op.apply_phi(Xd)), rtol=0, atol=1e-12 * np.abs(PX).max())


@pytest.mark.parametrize("reorth", [0, 1])
@pytest.mark.parametrize("nops", [2, 3])
def test_multi_lanczos_fp32_block16(ctx, lib, nops, reorth):
    """FP32 Lanczos groups of 16 columns (32 or 48 values per row; three groups take two
    workgroup column chunks in the grouped kernels), Barabasi-Albert n = 3000; reorth 0
    (projection against the current block only) and 1 (second local pass against the
    previous block too), grouped and single-operator paths alike."""
    print(f"[gpu] multi lanczos fp32 b16 nops={nops} reorth={reorth}", flush=True)
    n = 3000
    rp, ci = synth.barabasi_albert(n, 5, 13)
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    specs = [(0.5, "res", _res_alpha(g, 0.5, lam)), (1.0, "res", _res_alpha(g, 1.0, lam)),
             (0.0, "exp", 1.0 / lam)][:nops]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float32, krylov_dim=30, method="lanczos", reorth=reorth)
           for mu, f, p in specs]
    multi = lib.Multi(ops)
    X = synth.rademacher_block(n, 16, 3)
    Xd = dev(X, torch.float32)
    LX = host(multi.apply_L(Xd))
    W = host(multi.fdeg())
    for i, (op, (mu, f, p)) in enumerate(zip(ops, specs)):
        cols = slice(16 * i, 16 * (i + 1))
        wr = sparse.fdeg(As, mu, f, p)
        pr = sparse.phi_apply(As, mu, f, p, X)
        assert np.linalg.norm(W[:, i] - wr) < 2e-5 * np.linalg.norm(wr), (mu, f)
        scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(pr)
        assert np.linalg.norm(LX[:, cols] - (wr[:, None] * X - pr)) < 2e-5 * scale, (mu, f)
        assert np.linalg.norm(LX[:, cols] - host(op.apply_L(Xd))) < 2e-5 * scale, (mu, f)


def test_multi_lanczos_small_graph_full_reorth_fallback(ctx, lib):
    """(steps + 1) 2 b > n: every operator runs alone (full reorthogonalisation), and the
    grouped result equals the single operators'."""
    print("[gpu] multi lanczos small graph", flush=True)
    n = 90
    rp, ci = synth.erdos_renyi_gnm(n, 400, 4)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    ops = [lib.Operator(g, mu, "res", 0.5 / lam, dtype=torch.float64, krylov_dim=20, method="lanczos")
           for mu in (0.0, 0.25)]
    multi = lib.Multi(ops)
    X = synth.gaussian_block(n, 16, 9)
    Xd = dev(X, torch.float64)
    PX = host(multi.apply_phi(Xd))
    for i, (op, mu) in enumerate(zip(ops, (0.0, 0.25))):
        ph = genfun.phi(A, mu, "res", 0.5 / lam)
        cols = slice(16 * i, 16 * (i + 1))
        assert np.linalg.norm(PX[:, cols] - ph @ X) < 1e-8 * np.linalg.norm(ph @ X)
        np.testing.assert_allclose(PX[:, cols], host(op.apply_phi(Xd)), rtol=0, atol=1e-12 * np.abs(PX).max())


def test_multi_fp32_narrow_rows_per_column_weights(ctx, lib):
    """Five series operators with one column each (rows of 5 FP32 values held by one
    lane, every column with its own operator's weights and finish): walk degrees and
    L x against the single operators."""
    print("[gpu] multi fp32 narrow rows", flush=True)
    n = 5000
    rp, ci = synth.barabasi_albert(n, 4, 17)
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    mus = [0.0, 0.25, 0.5, 0.75, 1.0]
    ops = [lib.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=20 + 2 * i)
           for i, mu in enumerate(mus)]
    multi = lib.Multi(ops)
    W = host(multi.fdeg())
    x = synth.gaussian_block(n, 1, 8)
    LX = host(multi.apply_L(dev(x, torch.float32)))
    for i, (op, mu) in enumerate(zip(ops, mus)):
        wr = sparse.fdeg(As, mu, "exp", 1.0 / lam)
        assert np.linalg.norm(W[:, i] - wr) < 1e-5 * np.linalg.norm(wr), mu
        assert np.linalg.norm(W[:, i] - host(op.fdeg())) < 1e-6 * np.linalg.norm(wr), mu
        pr = sparse.phi_apply(As, mu, "exp", 1.0 / lam, x)
        scale = np.linalg.norm(wr[:, None] * x) + np.linalg.norm(pr)
        assert np.linalg.norm(LX[:, i] - (wr * x[:, 0] - pr[:, 0])) < 2e-5 * scale, mu


def test_multi_lanczos_fp32_rank_deficient_block(ctx, lib):
    """A 16-wide start block of rank 10 (six columns repeat others): every group
    deflates the repeated directions in its first CholQR and still reproduces phi X
    column by column (repeated columns give repeated results)."""
    print("[gpu] multi lanczos rank-deficient block", flush=True)
    n = 3000
    rp, ci = synth.barabasi_albert(n, 5, 19)
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    specs = [(0.5, "res", _res_alpha(g, 0.5, lam)), (0.0, "exp", 1.0 / lam)]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float32, krylov_dim=30, method="lanczos") for mu, f, p in specs]
    multi = lib.Multi(ops)
    X = synth.gaussian_block(n, 16, 23)
    X[:, 10:] = X[:, :6]
    Xd = dev(X, torch.float32)
    PX = host(multi.apply_phi(Xd))
    for i, (mu, f, p) in enumerate(specs):
        pr = sparse.phi_apply(As, mu, f, p, X)
        cols = slice(16 * i, 16 * (i + 1))
        assert np.linalg.norm(PX[:, cols] - pr) < 2e-5 * np.linalg.norm(pr), (mu, f)
        assert np.linalg.norm(PX[:, cols][:, 10:] - PX[:, cols][:, :6]) < 2e-5 * np.linalg.norm(pr), (mu, f)


def test_multi_lanczos_nine_single_columns_fall_back(ctx, lib):
    """Nine single-column Lanczos groups exceed the grouped kernels' eight: the walk
    degrees are evaluated operator by operator and equal the single operators'."""
    print("[gpu] multi lanczos nine groups", flush=True)
    n = 500
    rp, ci = synth.erdos_renyi_gnm(n, 2500, 31)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    mus = np.linspace(0.0, 1.0, 9)
    ops = [lib.Operator(g, mu, "res", _res_alpha(g, mu, lam), dtype=torch.float64, krylov_dim=40, method="lanczos")
           for mu in mus]
    W = host(lib.Multi(ops).fdeg())
    for i, (op, mu) in enumerate(zip(ops, mus)):
        w = genfun.phi(A, mu, "res", _res_alpha(g, mu, lam)).sum(1)
        assert np.linalg.norm(W[:, i] - w) < 1e-8 * np.linalg.norm(w), mu
        np.testing.assert_allclose(W[:, i], host(op.fdeg()), rtol=0, atol=1e-13 * np.abs(w).max())


def test_multi_lanczos_rank_deficient_block_small_graph(ctx, lib):
    """A start block of rank 4 in 16 columns on a 99-node lattice with many components
    (edges kept w.p. 0.35), FP64, resolvent (mu = 1) and exponential (mu = 0) side by
    side with 30 steps: the block Krylov space grows by 4 per step, so the runs must not
    stop at the full-rank step count n / 16 + 1 (8); phi X against the dense phi to
    1e-10."""
    print("[gpu] multi lanczos rank-deficient block on a small disconnected graph", flush=True)
    rp, ci = synth.road_grid(9, 11, 0.35, seed=11)
    n = len(rp) - 1
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    specs = [(1.0, "res", 0.5 / g.spectral_radius(1.0)), (0.0, "exp", 1.0 / lam)]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float64, krylov_dim=30, method="lanczos", tol=1e-14)
           for mu, f, p in specs]
    multi = lib.Multi(ops)
    X = synth.gaussian_block(n, 16, 31)
    X[:, 4:] = X[:, :4] @ np.random.default_rng(3).standard_normal((4, 12))
    PX = host(multi.apply_phi(dev(X, torch.float64)))
    for i, (mu, f, p) in enumerate(specs):
        pr = sparse.phi_apply(As, mu, f, p, X)
        cols = slice(16 * i, 16 * (i + 1))
        err = np.linalg.norm(PX[:, cols] - pr) / np.linalg.norm(pr)
        print(f"[gpu]   {f} mu={mu}: relative error {err:.2e}", flush=True)
        assert err < 1e-10, (mu, f, err)
