"""The learned control variate's device kernels against the oracle: features,
exact diagonals, MLP forward / backward / Adam, and the control-variate estimator."""

import numpy as np
import pytest

import synth
from oracle import estimators, features, genfun, mlp, philox, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def test_features_match_definitions(ctx, lib):
    for name, (n, rp, ci) in {"ba": (3000,) + synth.barabasi_albert(3000, 4, 1),
                              "sbm": (2000,) + synth.stochastic_block_model(2000, 8, 10, 20, 2),
                              "toy": (13,) + synth.toy_g58()}.items():
        print(f"[gpu] features {name}", flush=True)
        g = lib.Graph(ctx, rp, ci)
        f = g.features(0.05).cpu().numpy().astype(np.float64)
        ref = features.features(n, rp, ci, 0.05)
        np.testing.assert_allclose(f, ref, rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("mu,kind", [(0.0, "res"), (0.5, "exp"), (1.0, "res")])
def test_diag_exact(ctx, lib, dtype, tol, mu, kind):
    n = 500
    rp, ci = synth.erdos_renyi_gnm(n, 2000, 4)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu)) if kind == "res" else 1.0 / lam
    td = torch.float64 if dtype == "f64" else torch.float32
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, kind, param, dtype=td, krylov_dim=40)
    nodes = np.array([0, 5, 17, 499, 250, 3, 77] + list(range(100, 140)), dtype=np.int32)
    got = op.diag_exact(nodes, width=16).cpu().numpy().astype(np.float64)
    ref = np.diag(genfun.phi(A, mu, kind, param))[nodes]
    np.testing.assert_allclose(got, ref, rtol=tol)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_mlp_forward_and_gradient_match_fp64_backprop(ctx, lib):
    p = f32(synth.glorot_params(mlp.SIZES, 3))
    N = 1000
    X = f32(synth.gaussian_block(N, 8, 4))
    t = f32(synth.gaussian_block(N, 1, 5)[:, 0])
    net = lib.MLP(ctx, p)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    y = net.forward(Xd).cpu().numpy().astype(np.float64)
    y_ref, _ = mlp.forward(p, X)
    np.testing.assert_allclose(y, y_ref, rtol=1e-5, atol=1e-5 * np.abs(y_ref).max())
    L, gr = net.loss_grad(Xd, td)
    L_ref, g_ref = mlp.loss_and_grad(p, X, t)
    assert abs(L - L_ref) < 1e-5 * L_ref
    np.testing.assert_allclose(gr, g_ref, rtol=1e-4, atol=1e-5 * np.abs(g_ref).max())


def test_mlp_adam_step_matches_oracle(ctx, lib):
    p = f32(synth.glorot_params(mlp.SIZES, 7))
    N = 512
    X = f32(synth.gaussian_block(N, 8, 8))
    t = f32(synth.gaussian_block(N, 1, 9)[:, 0])
    net = lib.MLP(ctx, p)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    td = torch.tensor(t, dtype=torch.float32, device="cuda")
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    pr = p.copy()
    for step in range(1, 4):
        net.train_step(Xd, td, 1e-3)
        _, g = mlp.loss_and_grad(pr, X, t)
        pr, m, v = mlp.adam_step(pr, g, m, v, step, 1e-3)
        pr = f32(pr)
    np.testing.assert_allclose(net.params().astype(np.float64), pr, atol=2e-6)


def test_mlp_save_load_roundtrip(ctx, lib, tmp_path):
    p = f32(synth.glorot_params(mlp.SIZES, 11))
    net = lib.MLP(ctx, p)
    path = tmp_path / "net.bin"
    net.save(path)
    net2 = lib.MLP.load_file(ctx, path)
    np.testing.assert_array_equal(net2.params(), net.params())


def test_training_reduces_loss_and_cv_helps(ctx, lib):
    """Train on exact diagonals of a few small graphs, then estimate diag phi on a
    held-out graph with 16 Gaussian probes (mean error over 10 seeds, normalised by
    ||diag phi - 1||) with: plain Hutchinson, the learned control variate, the trivial
    control variate g = 1, the exact diagonal as control variate (the best any diagonal
    predictor can do), BKS and Rademacher probes.
      * Against plain Gaussian Hutchinson the learned control variate gains more than 2x
        in error (4x in probes: the pass criterion of the learned part).
      * That gain is the trivial one: g = 1 removes the same omega_i^2 fluctuation.  A
        diagonal control variate leaves the off-diagonal noise sum_k F_ik^2, which
        dominates here, so even the exact diagonal is within 10 % of g = 1, and the
        learned network is no worse than g = 1 (within 5 %).  At these weights no learned
        gain exists over the best estimator without it (BKS and Rademacher are at the
        level of g = 1; the errors are printed)."""
    feats, targs = [], []
    for seed in range(6):
        n = 1500
        rp, ci = synth.barabasi_albert(n, 3 + seed % 3, 100 + seed)
        g = lib.Graph(ctx, rp, ci)
        lam = g.lambda_max()
        alpha = 0.5 / lam
        op = lib.Operator(g, 0.0, "res", alpha, dtype=torch.float32, krylov_dim=30)
        nodes = np.arange(n, dtype=np.int32)
        feats.append(g.features(alpha))
        targs.append(op.diag_exact(nodes, width=64) - 1.0)
    F = torch.cat(feats).contiguous()
    T = torch.cat(targs).contiguous()
    net = lib.MLP(ctx, synth.glorot_params(mlp.SIZES, 1))
    first = net.train_step(F, T, 3e-3)
    for _ in range(400):
        last = net.train_step(F, T, 3e-3)
    assert last < 0.2 * first
    # held-out graph
    n = 3000
    rp, ci = synth.barabasi_albert(n, 4, 999)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    lam = g.lambda_max()
    alpha = 0.5 / lam
    ph = genfun.phi(A, 0.0, "res", alpha)
    d = np.diag(ph)
    ghat = net.forward(g.features(alpha)).cpu().numpy().astype(np.float64) + 1.0
    errs = {k: [] for k in ("plain", "learned", "const", "exact", "bks", "rademacher")}
    den = np.linalg.norm(d - 1)
    for s in range(10):
        Om = philox.gaussian(n, 16, 500 + s)
        Y = ph @ Om
        errs["plain"].append(np.linalg.norm(estimators.hutchinson_diag(Om, Y) - d) / den)
        errs["learned"].append(np.linalg.norm(estimators.cv_diag(Om, Y, ghat) - d) / den)
        errs["const"].append(np.linalg.norm(estimators.cv_diag(Om, Y, np.ones(n)) - d) / den)
        errs["exact"].append(np.linalg.norm(estimators.cv_diag(Om, Y, d) - d) / den)
        errs["bks"].append(np.linalg.norm(estimators.bks_diag(Om, Y) - d) / den)
        R = philox.rademacher(n, 16, 500 + s)
        errs["rademacher"].append(np.linalg.norm(estimators.hutchinson_diag(R, ph @ R) - d) / den)
    e = {k: float(np.mean(v)) for k, v in errs.items()}
    print("[gpu] held-out diagonal errors, M = 16: " + ", ".join(f"{k} {v:.3g}" for k, v in e.items()), flush=True)
    assert e["learned"] < 0.5 * e["plain"]
    assert e["exact"] > 0.9 * e["const"]
    assert e["learned"] < 1.05 * e["const"]


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-10), ("f32", 2e-5)])
@pytest.mark.parametrize("mu,kind", [(0.5, "exp"), (1.0, "res"), (0.0, "exp")])
def test_surrogate_terms_and_targets(ctx, lib, dtype, tol, mu, kind):
    """Degree-3 diagonal and remainder scale per node, and the residual training targets
    (diag phi - base) / scale, against the dense oracle."""
    from oracle import features as ofeat
    n = 500
    rp, ci = synth.erdos_renyi_gnm(n, 2500, 6)
    A = walks.adjacency(n, rp, ci)
    td = torch.float64 if dtype == "f64" else torch.float32
    g = lib.Graph(ctx, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    param = 1.0 / lam if kind == "exp" else 0.5 / lam
    op = lib.Operator(g, mu, kind, param, dtype=td, krylov_dim=40)
    base, scale = op.surrogate_diag()
    rb, rs = ofeat.surrogate_terms(A, mu, kind, param)
    np.testing.assert_allclose(base.cpu().numpy(), rb, rtol=tol)
    np.testing.assert_allclose(scale.cpu().numpy(), rs, rtol=tol)
    nodes = np.arange(0, n, 7, dtype=np.int32)
    tgt = op.surrogate_target(nodes, width=16).cpu().numpy().astype(np.float64)
    ref = (np.diag(genfun.phi(A, mu, kind, param))[nodes] - rb[nodes]) / rs[nodes]
    # in units of diag phi (~1) the error is that of diag phi itself (the FP32 / FP64
    # contract); the target divides it by the small scale
    err_phi = np.abs(tgt - ref) * rs[nodes]
    assert err_phi.max() <= (2e-5 if dtype == "f32" else 1e-10), err_phi.max()


def test_mlp_predict_is_affine_forward(ctx, lib):
    net = lib.MLP(ctx, synth.glorot_params(mlp.SIZES, 4))
    rng = np.random.default_rng(0)
    F = torch.tensor(rng.standard_normal((1000, 8)), dtype=torch.float32, device="cuda")
    base = torch.tensor(rng.standard_normal(1000), dtype=torch.float32, device="cuda")
    scale = torch.tensor(rng.random(1000), dtype=torch.float32, device="cuda")
    y = net.forward(F)
    p = net.predict(F, base, scale)
    np.testing.assert_allclose(p.cpu().numpy(), (base + scale * y).cpu().numpy(), rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(net.predict(F).cpu().numpy(), y.cpu().numpy(), rtol=0, atol=0)
