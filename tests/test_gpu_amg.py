"""Multigrid-preconditioned CG on the deformed Laplacian (WL_M_AMG_CG) through the C ABI
against the oracle: the solution of A_mu(alpha) y = x (direct sparse solve), the
residual contract of every column (relative 1e-9, Sec. 5.3), the hierarchy (level sizes
equal to the oracle's) and the iteration counts of the oracle's PCG with the same
hierarchy, on the alpha grid 10^e / rho(Z_mu), e in linspace(-3, -0.5, 4) (Sec. 5.3),
plus alpha rho(Z_mu) = 0.9 and 0.99 where the preconditioner matters."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg, sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FRACS = [float(f) for f in 10.0 ** np.linspace(-3, -0.5, 4)] + [0.9, 0.99]


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def graphs():
    rp, ci = synth.road_grid(60, 60, 0.7, seed=7)
    g1 = ("grid", len(rp) - 1, rp, ci)
    rp, ci = synth.barabasi_albert(3000, 5, 3)
    return [g1, ("ba", 3000, rp, ci)]


@pytest.mark.parametrize("gi", [0, 1])
@pytest.mark.parametrize("mu", [0.0, 0.5, 1.0])
def test_amg_cg_alpha_grid(ctx, lib, gi, mu):
    name, n, rp, ci = graphs()[gi]
    print(f"[gpu] amg-cg {name} mu={mu}", flush=True)
    Adj = sparse.adjacency(n, rp, ci)
    rho = sparse.rho_Z(Adj, mu)
    g = lib.Graph(ctx, rp, ci, validate=True)
    X = synth.gaussian_block(n, 5, 11)
    Xd = torch.tensor(X, dtype=torch.float64, device="cuda")
    for frac in FRACS:
        alpha = frac / rho
        op = lib.Operator(g, mu, "res", alpha, dtype=torch.float64, method="amg", rho_hint=rho)
        Y = op.apply_phi(Xd).cpu().numpy()
        info = op.amg_info()
        A = sp.csr_matrix(sparse.deformed(Adj, mu, alpha))
        c0 = 1.0 - mu * mu * alpha * alpha
        # every column meets the relative residual 1e-9 on A_mu y = x (y = phi x / c0)
        for c in range(X.shape[1]):
            res = np.linalg.norm(X[:, c] - A @ (Y[:, c] / c0)) / np.linalg.norm(X[:, c])
            assert res <= 1.0001e-9, (frac, c, res)
        ref = sparse.phi_res_apply(Adj, mu, alpha, X)
        assert np.linalg.norm(Y - ref) / np.linalg.norm(ref) < 1e-7, frac
        # the hierarchy and the iteration count are the oracle's
        levels = amg.hierarchy(A)
        assert info["rows"] == [lv[0].shape[0] for lv in levels], (frac, info["rows"])
        _, its = amg.pcg(A, X, levels, tol=1e-9)
        print(f"[gpu]   alpha rho = {frac:.4f}: levels {info['rows']}, iterations {info['iterations']} "
              f"(oracle per column {its.tolist()})", flush=True)
        assert abs(info["iterations"] - int(its.max())) <= 1, (frac, info["iterations"], its)


def test_amg_walk_degree_laplacian_and_diffusion(ctx, lib):
    """fdeg, L X and exp(-t L) U0 with the multigrid inner solve agree with the Lanczos
    resolvent to the solver tolerances."""
    name, n, rp, ci = graphs()[0]
    Adj = sparse.adjacency(n, rp, ci)
    mu = 1.0
    rho = sparse.rho_Z(Adj, mu)
    alpha = 0.9 / rho
    g = lib.Graph(ctx, rp, ci)
    opa = lib.Operator(g, mu, "res", alpha, dtype=torch.float64, method="amg", rho_hint=rho, tol=1e-12)
    opl = lib.Operator(g, mu, "res", alpha, dtype=torch.float64, method="lanczos", krylov_dim=150, rho_hint=rho)
    wa, wl_ = opa.fdeg().cpu().numpy(), opl.fdeg().cpu().numpy()
    wr = sparse.fdeg(Adj, mu, "res", alpha)
    assert np.max(np.abs(wa - wr) / wr) < 1e-9 and np.max(np.abs(wl_ - wr) / wr) < 1e-8
    X = torch.tensor(synth.gaussian_block(n, 3, 4), dtype=torch.float64, device="cuda")
    La, Ll = opa.apply_L(X).cpu().numpy(), opl.apply_L(X).cpu().numpy()
    assert np.linalg.norm(La - Ll) / np.linalg.norm(Ll) < 1e-8
    U0 = torch.tensor(synth.spike_block(n, [0, 17, 900]), dtype=torch.float64, device="cuda")
    (Ea,), _ = opa.expv(U0, [1.0], outer_dim=40)
    (El,), _ = opl.expv(U0, [1.0], outer_dim=40)
    assert torch.linalg.norm(Ea - El) / torch.linalg.norm(El) < 1e-8


def test_amg_rejections(ctx, lib):
    name, n, rp, ci = graphs()[1]
    g = lib.Graph(ctx, rp, ci)
    with pytest.raises(lib.WLError, match="UNSUPPORTED"):
        lib.Operator(g, 0.5, "res", 0.001, dtype=torch.float32, method="amg")
    with pytest.raises(lib.WLError, match="UNSUPPORTED"):
        lib.Operator(g, 0.0, "exp", 0.01, dtype=torch.float64, method="amg")
    # near the pole (alpha rho(Z) = 0.99) one preconditioned iteration cannot reach 1e-14;
    # at alpha = 0.001 the deformed Laplacian is so close to the identity that one
    # iteration may already meet it
    rho = sparse.rho_Z(sparse.adjacency(n, rp, ci), 0.5)
    op = lib.Operator(g, 0.5, "res", 0.99 / rho, dtype=torch.float64, method="amg", krylov_dim=1, tol=1e-14,
                      rho_hint=rho)
    X = torch.tensor(synth.gaussian_block(n, 2, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.WLError, match="ENOCONV"):
        op.apply_phi(X)
