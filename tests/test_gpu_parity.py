"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Tolerances (relative):
  * FP64 path: 1e-8 for every output (L X measured against ||w*X|| + ||phi X||,
    since L X cancels: L 1 = 0).
  * FP32 path: w 1e-5; phi X and L X 2e-5 (same normalisation); diffusion 1e-4.
These follow from FP32 storage (unit roundoff 6e-8) amplified by at most ~30
recurrence / Lanczos steps with FP64 coefficients and inner products.
"""

import numpy as np
import pytest

import synth
from oracle import estimators, genfun, laplacian, philox, sparse, walks

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def wl(lib):
    return lib


@pytest.fixture(scope="module")
def ctx(wl):
    print("[gpu] creating context", flush=True)
    return wl.Context(0)


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b, scale=None):
    s = np.linalg.norm(b) if scale is None else scale
    return np.linalg.norm(a - b) / max(s, 1e-300)


def node_rel(a, b, mag):
    """Largest error of any node (and column) against that node's magnitude mag (n, or
    n x b): the norm-wise checks alone would let hub rows hide errors on the many
    low-degree nodes."""
    mag = np.asarray(mag, dtype=np.float64)
    if mag.ndim == 1 and np.ndim(a) == 2:
        mag = mag[:, None]
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)) / np.maximum(mag, 1e-300)))


# ------------------------------------------------------------------ SpMM
def spmm_graphs():
    star_iso = synth.csr_from_edges(3000, np.zeros(2500, dtype=np.int64), np.arange(1, 2501))  # hub + isolated
    return {
        "er": (500,) + synth.erdos_renyi_gnm(500, 2000, 3),
        "ba": (6000,) + synth.barabasi_albert(6000, 5, 4),
        "star_iso": (3000,) + star_iso,
        "cycle": (257,) + synth.cycle_graph(257),
    }


@pytest.mark.parametrize("gname", ["er", "ba", "star_iso", "cycle"])
@pytest.mark.parametrize("b", [1, 2, 3, 5, 7, 8, 12, 16, 20, 24, 28, 32, 40, 48, 60, 64, 96])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_spmm_matches_sparse_product(ctx, wl, gname, b, dtype):
    n, rp, ci = spmm_graphs()[gname]
    print(f"[gpu] spmm {gname} b={b} {dtype}", flush=True)
    td = torch.float32 if dtype == "f32" else torch.float64
    g = wl.Graph(ctx, rp, ci, validate=True)
    X = synth.gaussian_block(n, b, 7)
    Y = host(g.spmm(dev(X, td)))
    ref = sparse.adjacency(n, rp, ci) @ X
    tol = 2e-6 if dtype == "f32" else 1e-14
    assert rel(Y, ref) < tol


def test_spmm_autotuned_shape_same_result(ctx, wl):
    n, rp, ci = spmm_graphs()["ba"]
    g = wl.Graph(ctx, rp, ci)
    X = dev(synth.gaussian_block(n, 16, 1), torch.float32)
    before = host(g.spmm(X))
    g.autotune(torch.float32, 16)
    after = host(g.spmm(X))
    ref = sparse.adjacency(n, rp, ci) @ host(X)
    assert rel(after, ref) < 2e-6 and rel(before, ref) < 2e-6


@pytest.mark.parametrize("G", [1, 4, 16, 64])
def test_spmm_explicit_shape_same_result(ctx, wl, G):
    n, rp, ci = spmm_graphs()["ba"]
    g = wl.Graph(ctx, rp, ci)
    g.set_shape(torch.float32, 16, G, 8)
    got_g, got_thr = g.shape(torch.float32, 16)
    assert got_g == max(G, 4) and got_thr >= 8
    X = dev(synth.gaussian_block(n, 16, 2), torch.float32)
    ref = sparse.adjacency(n, rp, ci) @ host(X)
    assert rel(host(g.spmm(X)), ref) < 2e-6


# ------------------------------------------------------------------ FP64, dense oracle
def er_small():
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    return n, rp, ci, walks.adjacency(n, rp, ci)


@pytest.mark.parametrize("mu", [0.0, 0.25, 0.5, 0.75, 1.0])
@pytest.mark.parametrize("kind", ["res", "exp"])
def test_fp64_variants_match_dense(ctx, wl, mu, kind):
    n, rp, ci, A = er_small()
    print(f"[gpu] fp64 variant mu={mu} {kind}", flush=True)
    g = wl.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu)) if kind == "res" else 1.0 / lam
    op = wl.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=40)
    ph = genfun.phi(A, mu, kind, param)
    X = synth.gaussian_block(n, 5, 3)
    w = host(op.fdeg())
    PX = host(op.apply_phi(dev(X, torch.float64)))
    LX = host(op.apply_L(dev(X, torch.float64)))
    wr = laplacian.walk_degree(ph)
    assert rel(w, wr) < 1e-8
    assert rel(PX, ph @ X) < 1e-8
    scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(ph @ X)
    assert rel(LX, laplacian.apply_laplacian(ph, X), scale) < 1e-8
    # per node: w against itself, phi X against |phi| |X| (the size of the sum it is)
    mag = np.abs(ph) @ np.abs(X)
    assert node_rel(w, wr, wr) < 1e-8
    assert node_rel(PX, ph @ X, mag) < 1e-8
    assert node_rel(LX, laplacian.apply_laplacian(ph, X), np.abs(wr)[:, None] * np.abs(X) + mag) < 1e-8


def test_mu0_exponential_lanczos_matches_dense(ctx, wl):
    n, rp, ci, A = er_small()
    g = wl.Graph(ctx, rp, ci)
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    op = wl.Operator(g, 0.0, "exp", beta, dtype=torch.float64, krylov_dim=30, method="lanczos")
    X = synth.gaussian_block(n, 4, 5)
    ph = genfun.phi(A, 0.0, "exp", beta)
    assert rel(host(op.apply_phi(dev(X, torch.float64))), ph @ X) < 1e-8


def test_config1_er1000_fp64(ctx, wl):
    """ER n=1000, mean degree 8, resolvent mu=0 alpha=0.5/lambda_max, FP64:
    f(A)1, L x (Gaussian x), exp(-L) e_0."""
    n = 1000
    rp, ci = synth.erdos_renyi_gnm(n, 4000, 1)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    alpha = 0.5 / lam
    g = wl.Graph(ctx, rp, ci, validate=True)
    assert abs(g.lambda_max() - lam) < 1e-10 * lam
    op = wl.Operator(g, 0.0, "res", alpha, dtype=torch.float64, krylov_dim=40)
    ph = genfun.phi(A, 0.0, "res", alpha)
    L = laplacian.walk_laplacian(ph)
    x = synth.gaussian_block(n, 1, 2)
    u0 = synth.spike_block(n, [0])
    w = host(op.fdeg())
    Lx = host(op.apply_L(dev(x, torch.float64)))
    (Y,), err = op.expv(dev(u0, torch.float64), [1.0], outer_dim=30)
    wr = ph.sum(1)
    assert rel(w, wr) < 1e-8
    assert rel(Lx, L @ x, np.linalg.norm(wr[:, None] * x) + np.linalg.norm(ph @ x)) < 1e-8
    (Yr,) = laplacian.expv(L, u0, [1.0])
    assert rel(host(Y), Yr) < 1e-8
    assert err[0] < 1e-8


# ------------------------------------------------------------------ FP32, sparse oracle
@pytest.fixture(scope="module")
def ba_mid():
    n = 20000
    rp, ci = synth.barabasi_albert(n, 5, 11)
    return n, rp, ci, sparse.adjacency(n, rp, ci)


@pytest.mark.parametrize("mu", [0.0, 0.25, 0.5, 0.75, 1.0])
@pytest.mark.parametrize("kind", ["exp", "res"])
def test_fp32_block16_k30_matches_oracle(ctx, wl, ba_mid, mu, kind):
    n, rp, ci, As = ba_mid
    print(f"[gpu] fp32 BA20k mu={mu} {kind}", flush=True)
    g = wl.Graph(ctx, rp, ci)
    lam = sparse.lambda_max(As)
    param = 1.0 / lam if kind == "exp" else 0.5 / sparse.rho_Z(As, mu)
    op = wl.Operator(g, mu, kind, param, dtype=torch.float32, krylov_dim=30)
    X = synth.rademacher_block(n, 16, 3)
    w = host(op.fdeg())
    PX = host(op.apply_phi(dev(X, torch.float32)))
    LX = host(op.apply_L(dev(X, torch.float32)))
    wr = sparse.fdeg(As, mu, kind, param)
    pr = sparse.phi_apply(As, mu, kind, param, X)
    assert rel(w, wr) < 1e-5
    assert rel(PX, pr) < 2e-5
    scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(pr)
    assert rel(LX, wr[:, None] * X - pr, scale) < 2e-5
    # per node: phi >= 0 entrywise (weights and walk counts are nonnegative), so for
    # Rademacher X the size of (phi X)_ij is at most (phi |X|)_i = w_i, and of (L X)_ij
    # at most 2 w_i
    ew, ep, el = node_rel(w, wr, wr), node_rel(PX, pr, wr), node_rel(LX, wr[:, None] * X - pr, 2 * wr)
    print(f"[gpu] per-node errors: w {ew:.1e}, phi X {ep:.1e}, L X {el:.1e}", flush=True)
    assert ew < 2e-5 and ep < 1e-4 and el < 1e-4


# ------------------------------------------------------------------ spectral scale
def test_lambda_max_and_rho_z(ctx, wl):
    n = 3000
    rp, ci = synth.barabasi_albert(n, 4, 2)
    As = sparse.adjacency(n, rp, ci)
    g = wl.Graph(ctx, rp, ci)
    lam = sparse.lambda_max(As)
    assert abs(g.lambda_max() - lam) < 1e-9 * lam
    for mu in (0.25, 0.5, 1.0):
        r = sparse.rho_Z(As, mu)
        assert abs(g.spectral_radius(mu) - r) < 1e-7 * r, mu


def test_rho_z_regular_closed_form(ctx, wl):
    n, d = 64, 6
    rp, ci = synth.circulant_graph(n, [1, 2, 5])
    g = wl.Graph(ctx, rp, ci)
    for mu in (0.0, 0.5, 1.0):
        assert abs(g.spectral_radius(mu) - (d - mu)) < 1e-8 * d


# ------------------------------------------------------------------ probes
@pytest.mark.parametrize("shape", [(1000, 16), (333, 7), (5, 3)])
def test_probes_match_oracle_philox(ctx, wl, shape):
    n, M = shape
    r = host(wl.probes(ctx, n, M, seed=0x1234ABCD5678, law="rademacher", dtype=torch.float32))
    np.testing.assert_array_equal(r, philox.rademacher(n, M, 0x1234ABCD5678))
    gd = host(wl.probes(ctx, n, M, seed=99, law="gauss", dtype=torch.float64))
    np.testing.assert_allclose(gd, philox.gaussian(n, M, 99), rtol=1e-13, atol=1e-13)
    gf = host(wl.probes(ctx, n, M, seed=99, law="gauss", dtype=torch.float32))
    np.testing.assert_allclose(gf, philox.gaussian(n, M, 99), rtol=1.2e-7, atol=1e-7)


# ------------------------------------------------------------------ estimators
def spd_target(n, seed):
    rp, ci = synth.erdos_renyi_gnm(n, 3 * n, seed)
    A = walks.adjacency(n, rp, ci)
    L = laplacian.walk_laplacian(genfun.phi(A, 0.5, "exp", 1.0 / np.linalg.eigvalsh(A)[-1]))
    lamv, V = np.linalg.eigh(L)
    return (V * np.exp(-0.7 * lamv)) @ V.T


@pytest.mark.parametrize("M", [4, 16, 33])
def test_estimators_match_oracle(ctx, wl, M):
    n = 300
    F = spd_target(n, 5)
    Om = philox.gaussian(n, M, 17)
    Y = F @ Om
    g = np.abs(np.diag(F)) * 0.9
    Omd, Yd = dev(Om, torch.float64), dev(Y, torch.float64)
    d, tr, te = wl.estimate(ctx, Omd, Yd, "hutchinson")
    np.testing.assert_allclose(host(d), estimators.hutchinson_diag(Om, Y), rtol=1e-12)
    assert abs(tr - estimators.hutchinson_trace(Om, Y)) < 1e-10 * abs(tr)
    d, _, _ = wl.estimate(ctx, Omd, Yd, "bks")
    np.testing.assert_allclose(host(d), estimators.bks_diag(Om, Y), rtol=1e-12)
    d, _, _ = wl.estimate(ctx, Omd, Yd, "hutchinson", cv=dev(g, torch.float64))
    np.testing.assert_allclose(host(d), estimators.cv_diag(Om, Y, g), rtol=1e-12, atol=1e-14)
    d, tr, te = wl.estimate(ctx, Omd, Yd, "xnys", rcond=1e-10)
    t_o, e_o, d_o, _ = estimators.xnys(Om, Y, rcond=1e-10)
    assert abs(tr - t_o) < 1e-9 * abs(t_o)
    assert abs(te - e_o) < 1e-6 * abs(e_o) + 1e-12
    np.testing.assert_allclose(host(d), d_o, rtol=1e-8, atol=1e-10 * np.abs(d_o).max())


@pytest.mark.parametrize("M", [16, 20, 32, 64])
def test_estimators_fp32_matrix_core_gram(ctx, wl, M):
    """FP32 blocks take the matrix-core Gram (FP64 accumulation); widths that are not
    a multiple of 16 are padded.  Inputs are FP32-representable, so the oracle sees
    exactly the GPU's inputs."""
    n = 5000
    rng = np.random.default_rng(M)
    G = rng.standard_normal((n, 12)).astype(np.float32).astype(np.float64)
    Om = philox.gaussian(n, M, 3).astype(np.float32).astype(np.float64)
    Y = ((G @ (G.T @ Om)) / n + 0.5 * Om).astype(np.float32).astype(np.float64)
    Omd, Yd = dev(Om, torch.float32), dev(Y, torch.float32)
    _, tr, te = wl.estimate(ctx, Omd, Yd, "hutchinson", want_diag=False)
    assert abs(tr - estimators.hutchinson_trace(Om, Y)) < 1e-9 * abs(tr)
    d, tr, te = wl.estimate(ctx, Omd, Yd, "xnys", rcond=1e-9)
    t_o, e_o, d_o, _ = estimators.xnys(Om, Y, rcond=1e-9)
    assert abs(tr - t_o) < 1e-7 * abs(t_o)
    np.testing.assert_allclose(host(d), d_o, rtol=2e-5, atol=2e-5 * np.abs(d_o).max())


def test_xnys_low_rank_exact_on_gpu(ctx, wl):
    n, r, M = 200, 3, 8
    G = synth.gaussian_block(n, r, 2)
    F = G @ G.T
    Om = philox.gaussian(n, M, 4)
    d, tr, te = wl.estimate(ctx, dev(Om, torch.float64), dev(F @ Om, torch.float64), "xnys", rcond=1e-12)
    assert abs(tr - np.trace(F)) < 1e-9 * np.trace(F)
    np.testing.assert_allclose(host(d), np.diag(F), atol=1e-9 * np.trace(F))


# ------------------------------------------------------------------ error paths and edge cases
def test_error_paths(ctx, wl):
    n, rp, ci, A = er_small()
    g = wl.Graph(ctx, rp, ci)
    rho = walks.spectral_radius(walks.linearisation(A, 1.0))
    with pytest.raises(wl.WLError) as e:
        wl.Operator(g, 1.0, "res", 1.01 / rho, dtype=torch.float64)
    assert e.value.status == wl._lib.WL_ERANGE
    with pytest.raises(wl.WLError) as e:
        wl.Operator(g, 0.5, "exp", 0.1, method="lanczos")
    assert e.value.status == wl._lib.WL_EUNSUPPORTED
    with pytest.raises(wl.WLError) as e:
        wl.Operator(g, 1.5, "exp", 0.1)
    assert e.value.status == wl._lib.WL_EINVAL
    # asymmetric CSR is rejected with validation
    bad_rp = np.array([0, 1, 1], dtype=np.int32)
    bad_ci = np.array([1], dtype=np.int32)
    with pytest.raises(wl.WLError) as e:
        wl.Graph(ctx, bad_rp, bad_ci, validate=True)
    assert e.value.status == wl._lib.WL_EINVAL
    # a column out of range is rejected even without validation
    with pytest.raises(wl.WLError):
        wl.Graph(ctx, np.array([0, 1, 2], dtype=np.int32), np.array([1, 7], dtype=np.int32))
    # rowptr inconsistent with nnz
    with pytest.raises(wl.WLError):
        wl.Graph(ctx, np.array([0, 1, 3], dtype=np.int32), np.array([1, 0], dtype=np.int32))


def test_edgeless_and_tiny_graphs(ctx, wl):
    # no edges: phi = I for both families, L = 0
    rp = np.zeros(6, dtype=np.int32)
    ci = np.zeros(0, dtype=np.int32)
    g = wl.Graph(ctx, rp, ci, validate=True)
    for kind, param in (("exp", 0.3), ("res", 0.3)):
        op = wl.Operator(g, 0.5, kind, param, dtype=torch.float64, krylov_dim=5)
        np.testing.assert_allclose(host(op.fdeg()), np.ones(5), atol=1e-14)
        X = synth.gaussian_block(5, 2, 1)
        np.testing.assert_allclose(host(op.apply_L(dev(X, torch.float64))), 0, atol=1e-14)
    # Fig. 1 toy graph: Krylov space exhausted before K (deflation), resolvent + exponential
    rp, ci = synth.toy_g58()
    A = walks.adjacency(13, rp, ci)
    g = wl.Graph(ctx, rp, ci, validate=True)
    lam = np.linalg.eigvalsh(A)[-1]
    for mu, kind, param in [(0.0, "res", 1 / (2 * lam)), (0.0, "exp", 1.0), (1.0, "exp", 1.0), (1.0, "res", 0.2)]:
        op = wl.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=30)
        w = host(op.fdeg())
        np.testing.assert_allclose(w, genfun.phi(A, mu, kind, param).sum(1), rtol=1e-10)


@pytest.mark.parametrize("n,m,b", [(13, None, 8), (200, 900, 8), (60, 200, 16)])
def test_fp32_krylov_space_exhausted(ctx, wl, n, m, b):
    """FP32 graphs smaller than the Krylov dimension (n < K b, n not a multiple of b):
    the last block is partly rounding noise and must be deflated, not normalised.
    apply_L (resolvent, Lanczos) 2e-5 and diffusion 1e-4 against the dense oracle."""
    print(f"[gpu] exhausted Krylov space n={n} b={b}", flush=True)
    if m is None:
        rp, ci = synth.toy_g58()
    else:
        rp, ci = synth.erdos_renyi_gnm(n, m, 12)
    A = walks.adjacency(n, rp, ci)
    g = wl.Graph(ctx, rp, ci, validate=True)
    lam = np.linalg.eigvalsh(A)[-1]
    X = synth.gaussian_block(n, b, 3).astype(np.float32).astype(np.float64)
    for mu, kind, param in [(0.5, "res", 0.5 / lam), (0.25, "exp", 1.0 / lam)]:
        ph = genfun.phi(A, mu, kind, param)
        op = wl.Operator(g, mu, kind, param, dtype=torch.float32, krylov_dim=30)
        Y = host(op.apply_L(dev(X, torch.float32)))
        ref = laplacian.apply_laplacian(ph, X)
        scale = np.linalg.norm(ph.sum(1)[:, None] * X) + np.linalg.norm(ph @ X)
        assert np.linalg.norm(Y - ref) < 2e-5 * scale, (mu, kind)
        L = laplacian.walk_laplacian(ph)
        outs, _ = op.expv(dev(X, torch.float32), [0.1, 1.0, 10.0], outer_dim=30)
        for t, o in zip([0.1, 1.0, 10.0], outs):
            (r,) = laplacian.expv(L, X, [t])
            assert np.linalg.norm(host(o) - r) < 1e-4 * np.linalg.norm(r), (mu, kind, t)


def test_fp64_lanczos_spanning_the_space(ctx, wl):
    """FP64 block Lanczos whose basis spans most of the space (K b > n): every block is
    orthogonalised against all earlier ones, so the projection stays exact (1e-8)."""
    print("[gpu] fp64 Lanczos spanning the space", flush=True)
    n = 300
    rp, ci = synth.erdos_renyi_gnm(n, 1200, 8)
    A = walks.adjacency(n, rp, ci)
    g = wl.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    X = synth.gaussian_block(n, 24, 2)
    for mu, kind, param, method in [(0.5, "res", 0.5 / lam, "lanczos"), (0.0, "exp", 1.0 / lam, "lanczos")]:
        op = wl.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=30, method=method, tol=1e-13)
        ph = genfun.phi(A, mu, kind, param)
        assert rel(host(op.apply_phi(dev(X, torch.float64))), ph @ X) < 1e-8, (mu, kind)
        L = laplacian.walk_laplacian(ph)
        outs, _ = op.expv(dev(X, torch.float64), [1.0], outer_dim=30)
        (r,) = laplacian.expv(L, X, [1.0])
        assert rel(host(outs[0]), r) < 1e-8, (mu, kind)


def test_fig1_stationary_from_gpu_fdeg(ctx, wl):
    """The printed Fig. 1 bars follow from the GPU walk degree: pi = w / sum(w)."""
    from test_oracle_genfun import load_fig1
    rp, ci = synth.toy_g58()
    g = wl.Graph(ctx, rp, ci)
    lam = 3.1964027540390294
    gold = load_fig1()
    for key, (mu, kind, param) in {"res": (0.0, "res", 1 / (2 * lam)), "exp": (0.0, "exp", 1.0)}.items():
        w = host(wl.Operator(g, mu, kind, param, dtype=torch.float64, krylov_dim=30).fdeg())
        pi = w / w.sum()
        for node, val in gold[key].items():
            assert abs(pi[node - 1] - val) < 1e-13
