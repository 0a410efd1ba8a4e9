"""wl_diag_est end to end (probes -> operator -> estimator) against the dense oracle,
including more probes than one 64-column block (blocks of 64 columns, block c drawn
from Philox stream c, row sums accumulated on the device).  FP64 operator: 1e-8
relative, as every FP64 output."""

import numpy as np
import pytest

import synth
from oracle import estimators, genfun, laplacian, philox, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def setup(lib):
    ctx = lib.Context(0)
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    A = walks.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci, validate=True)
    alpha = 0.5 / np.linalg.eigvalsh(A)[-1]
    op = lib.Operator(g, 0.5, "res", alpha, dtype=torch.float64, tol=1e-13)
    F = genfun.phi(A, 0.5, "res", alpha)
    return ctx, g, op, F, n, A, alpha


def probes(n, M, seed, law):
    draw = philox.gaussian if law == "gauss" else philox.rademacher
    if M <= 64:
        return draw(n, M, seed)
    return np.hstack([draw(n, min(64, M - 64 * c), seed, c) for c in range((M + 63) // 64)])


@pytest.mark.parametrize("M,est,law,use_cv", [
    (16, "hutchinson", "gauss", False),
    (16, "bks", "rademacher", False),
    (16, "hutchinson", "gauss", True),
    (16, "xnys", "gauss", False),
    (100, "hutchinson", "gauss", False),
    (100, "bks", "gauss", False),
    (200, "hutchinson", "rademacher", True),
    (16, "surrogate", "gauss", False),
    (16, "surrogate", "gauss", True),
    (100, "surrogate", "rademacher", True),
])
def test_diag_est_phi(setup, M, est, law, use_cv):
    ctx, g, op, F, n, A, alpha = setup
    print(f"[gpu] diag_est phi M={M} {est} {law} cv={use_cv}", flush=True)
    seed = 77
    Om = probes(n, M, seed, law)
    Y = F @ Om
    gcv = np.abs(np.diag(F)) * 0.95 if use_cv else None
    cv = torch.tensor(gcv, dtype=torch.float64, device="cuda") if use_cv else None
    d, tr, te = op.diag_est(M, seed, target="phi", law=law, estimator=est, cv=cv)
    d = d.cpu().numpy()
    if est == "xnys":
        t_o, e_o, ref, _ = estimators.xnys(Om, Y, rcond=1e-10)
        assert abs(tr - t_o) < 1e-8 * abs(t_o)
    elif est == "surrogate":
        G = genfun.phi_series(A, 0.5, genfun.coefficients("res", alpha, 3))
        Z = G @ Om
        ref = estimators.surrogate_diag(Om, Y, Z, np.diag(G), gcv)
        t_o = estimators.surrogate_trace(Om, Y, Z, np.diag(G))
        assert abs(tr - t_o) < 1e-8 * abs(t_o)
    elif use_cv:
        ref = estimators.cv_diag(Om, Y, gcv)
    elif est == "bks":
        ref = estimators.bks_diag(Om, Y)
    else:
        ref = estimators.hutchinson_diag(Om, Y)
    if est not in ("xnys", "surrogate"):
        per_probe = np.einsum("ij,ij->j", Om, Y)
        assert abs(tr - per_probe.mean()) < 1e-8 * abs(per_probe.mean())
        assert abs(te - per_probe.std(ddof=1) / np.sqrt(M)) < 1e-6 * te
    assert np.linalg.norm(d - ref) < 1e-8 * np.linalg.norm(ref)


def test_diag_est_return_probabilities(setup):
    ctx, g, op, F, n, A, alpha = setup
    print("[gpu] diag_est exp(-tL) xnys", flush=True)
    M, seed, t = 24, 5, 1.0
    Om = probes(n, M, seed, "gauss")
    L = laplacian.walk_laplacian(F)
    (Y,) = laplacian.expv(L, Om, [t])
    d, tr, te = op.diag_est(M, seed, target="L", t=t, law="gauss", estimator="xnys", outer_dim=40)
    t_o, e_o, ref, _ = estimators.xnys(Om, Y, rcond=1e-10)
    assert abs(tr - t_o) < 1e-8 * abs(t_o)
    assert np.linalg.norm(d.cpu().numpy() - ref) < 1e-8 * np.linalg.norm(ref)


def test_diag_est_rejects_bad_arguments(setup, lib):
    ctx, g, op, F, n, A, alpha = setup
    with pytest.raises(lib.WLError):
        op.diag_est(100, 1, estimator="xnys")
    with pytest.raises(lib.WLError):
        op.diag_est(5000, 1)
    with pytest.raises(lib.WLError):
        op.diag_est(0, 1)
    with pytest.raises(lib.WLError):
        op.diag_est(16, 1, target="L", estimator="surrogate")


def test_surrogate_exact_for_linear_weights(setup, lib):
    """Linear weights (phi = I + A): the degree-3 surrogate G = c_0 I + c_1 A is phi
    itself, so the surrogate estimator's probe noise vanishes and diag phi = 1, tr phi = n
    come out exactly."""
    ctx, g, _, _, n, A, _ = setup
    op = lib.Operator(g, 0.0, "linear", 1.0, dtype=torch.float64)
    d, tr, te = op.diag_est(16, 3, target="phi", estimator="surrogate")
    np.testing.assert_allclose(d.cpu().numpy(), 1.0, atol=1e-13)
    assert abs(tr - n) < 1e-10 * n and abs(te) < 1e-10
