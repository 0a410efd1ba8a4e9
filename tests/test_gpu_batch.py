"""Batched evaluation of many graphs (one launch per Krylov step) against the
per-graph dense oracle: walk Laplacian products, diffusion exp(-t L) U0, and the
Nystrom average return probability."""

import numpy as np
import pytest

import synth
from oracle import estimators, genfun, laplacian, philox, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def mixed_graphs():
    gs = [
        (300,) + synth.erdos_renyi_gnm(300, 1200, 1),
        (250,) + synth.barabasi_albert(250, 3, 2),
        (400,) + synth.stochastic_block_model(400, 4, 10, 20, 3),
        (350,) + synth.configuration_model_powerlaw(350, 2.5, 2, 18, 4),
        (13,) + synth.toy_g58(),
        (200,) + synth.erdos_renyi_gnm(200, 900, 5),
    ]
    variants = [(0.0, "res"), (0.5, "exp"), (1.0, "res"), (0.25, "exp"), (0.75, "res"), (1.0, "exp")]
    ts = [1.0, 0.1, 10.0, 1.0, 0.5, 10.0]
    return gs, variants, ts


def dense_phi(n, rp, ci, mu, kind):
    A = walks.adjacency(n, rp, ci)
    if kind == "exp":
        param = 1.0 / max(np.linalg.eigvalsh(A)[-1], 1e-12)
    else:
        param = 0.5 / walks.spectral_radius(walks.linearisation(A, mu))
    return param, genfun.phi(A, mu, kind, param)


@pytest.fixture(scope="module")
def setup(ctx, lib):
    gs, variants, ts = mixed_graphs()
    graphs, descs, phis = [], [], []
    for (n, rp, ci), (mu, kind) in zip(gs, variants):
        param, ph = dense_phi(n, rp, ci, mu, kind)
        graphs.append(lib.Graph(ctx, rp, ci, validate=True))
        descs.append({"mu": mu, "func": kind, "param": param})
        phis.append(ph)
    batch = lib.Batch(ctx, graphs, descs, tol=1e-12)
    return batch, phis, ts


def test_batch_apply_L(setup):
    batch, phis, _ = setup
    b = 8
    Xs = [synth.gaussian_block(ph.shape[0], b, 10 + i) for i, ph in enumerate(phis)]
    X = batch.pack([torch.tensor(x, dtype=torch.float32, device="cuda") for x in Xs])
    Y = batch.apply_L(X)
    for i, (ph, x, y) in enumerate(zip(phis, Xs, batch.unpack(Y))):
        ref = laplacian.apply_laplacian(ph, x.astype(np.float32).astype(np.float64))
        w = ph.sum(1)
        scale = np.linalg.norm(w[:, None] * x) + np.linalg.norm(ph @ x)
        err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / scale
        assert err < 2e-5, (i, err)


def test_batch_tile_order_does_not_change_results(setup):
    """The XCD-grouped tile order only permutes which workgroup handles which rows."""
    batch, phis, _ = setup
    X = batch.pack([torch.tensor(synth.gaussian_block(ph.shape[0], 8, 30 + i), dtype=torch.float32, device="cuda")
                    for i, ph in enumerate(phis)])
    batch.xcd_grouped = False
    Y0 = batch.apply_L(X)
    batch.xcd_grouped = True
    Y1 = batch.apply_L(X)
    batch.xcd_grouped = False
    assert torch.equal(Y0, Y1)


def test_batch_expv_and_return_probability(setup):
    batch, phis, ts = setup
    b = 8
    Oms = [philox.gaussian(ph.shape[0], b, 100 + i).astype(np.float32).astype(np.float64) for i, ph in enumerate(phis)]
    U0 = batch.pack([torch.tensor(o, dtype=torch.float32, device="cuda") for o in Oms])
    Y, p_hat, p_err = batch.expv(U0, ts, outer_dim=30)
    for i, (ph, om, y, t) in enumerate(zip(phis, Oms, batch.unpack(Y), ts)):
        L = laplacian.walk_laplacian(ph)
        (ref,) = laplacian.expv(L, om, [t])
        err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)
        assert err < 1e-4, (i, err)
        n = ph.shape[0]
        tr_o, e_o, _, _ = estimators.xnys(om, ref, rcond=1e-10)
        assert abs(p_hat[i] - tr_o / n) < 1e-4 * max(tr_o / n, 1e-3) + 1e-6, (i, p_hat[i], tr_o / n)
        # the estimate is close to the true average return probability
        exact = laplacian.average_return_probability(L, t)
        assert abs(p_hat[i] - exact) < 6 * max(p_err[i], 1e-3), (i, p_hat[i], exact, p_err[i])


def test_batch_graph_replays_match_eager(setup, lib):
    """The captured diffusion replays with new U0 contents and times; every replay, with
    eager batched work between replays, equals the eager call bit for bit (same kernels
    in the same order on their own scratch)."""
    batch, phis, ts = setup
    b = 8
    U0 = batch.pack([torch.tensor(philox.gaussian(ph.shape[0], b, 200 + i), dtype=torch.float32, device="cuda")
                     for i, ph in enumerate(phis)])
    Y = torch.empty_like(U0)
    gr = batch.graph(U0, Y, outer_dim=30)
    assert lib.load().wl_batch_destroy(batch.handle) == lib._lib.WL_EINVAL  # graph still alive
    Ye = torch.empty_like(U0)
    for r in range(3):
        print(f"[gpu] batch graph replay {r}", flush=True)
        fresh = batch.pack([torch.tensor(philox.gaussian(ph.shape[0], b, 300 + 10 * r + i), dtype=torch.float32,
                                         device="cuda") for i, ph in enumerate(phis)])
        U0.copy_(fresh)
        tr = [t * (1.0 + 0.5 * r) for t in ts]
        _, ph_e, pe_e = batch.expv(U0, tr, outer_dim=30, out=Ye)
        torch.cuda.synchronize()
        ph_g, pe_g = gr.launch(tr, want_trace=True)
        torch.cuda.synchronize()
        assert torch.equal(Y, Ye), r
        np.testing.assert_array_equal(ph_g, ph_e)
        np.testing.assert_array_equal(pe_g, pe_e)
    gr.close()


def test_batch_graph_xcd_grouped_capture_first(ctx, lib):
    """A fresh batch switched to the XCD-grouped tile order and captured before any eager
    run at that width: the tile map is built before capture starts, and every replay
    equals the eager call in the same tile order bit for bit."""
    print("[gpu] batch graph xcd-grouped capture", flush=True)
    gs, variants, ts = mixed_graphs()
    graphs, descs, phis = [], [], []
    for (n, rp, ci), (mu, kind) in zip(gs, variants):
        param, ph = dense_phi(n, rp, ci, mu, kind)
        graphs.append(lib.Graph(ctx, rp, ci))
        descs.append({"mu": mu, "func": kind, "param": param})
        phis.append(ph)
    batch = lib.Batch(ctx, graphs, descs, tol=1e-12)
    batch.xcd_grouped = True
    b = 8
    U0 = batch.pack([torch.tensor(philox.gaussian(ph.shape[0], b, 500 + i), dtype=torch.float32, device="cuda")
                     for i, ph in enumerate(phis)])
    Y = torch.empty_like(U0)
    gr = batch.graph(U0, Y, outer_dim=30)
    Ye = torch.empty_like(U0)
    for r in range(3):
        tr = [t * (1.0 + 0.25 * r) for t in ts]
        gr.launch(tr)
        torch.cuda.synchronize()
        Yg = Y.clone()
        batch.expv(U0, tr, outer_dim=30, out=Ye, want_trace=False)
        torch.cuda.synchronize()
        assert torch.equal(Yg, Ye), r
    for i, (ph, y, t) in enumerate(zip(phis, batch.unpack(Y), [t * 1.5 for t in ts])):
        om = batch.unpack(U0)[i].cpu().numpy().astype(np.float64)
        (ref,) = laplacian.expv(laplacian.walk_laplacian(ph), om, [t])
        err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)
        assert err < 1e-4, (i, err)
    gr.close()
    batch.close()


def test_batch_diffusion_on_hub_graphs(lib):
    """Power-law graphs with hubs (a few large, fast-converging Ritz values of L) and a
    block model in one batch: exp(-t L) U0 against the dense oracle at t = 1 and 10."""
    print("[gpu] batch hub graphs", flush=True)
    ctx = lib.Context(0)
    gs = [(3000,) + synth.configuration_model_powerlaw(3000, 2.5, 2, 55, 41),
          (2000,) + synth.stochastic_block_model(2000, 8, 10, 20, 42)]
    graphs, descs, phis = [], [], []
    for n, rp, ci in gs:
        A = walks.adjacency(n, rp, ci)
        lam = np.linalg.eigvalsh(A)[-1]
        graphs.append(lib.Graph(ctx, rp, ci))
        descs.append({"mu": 0.5, "func": "res", "param": 0.5 / lam, "rho_hint": lam})
        phis.append(genfun.phi(A, 0.5, "res", 0.5 / lam))
    batch = lib.Batch(ctx, graphs, descs, tol=1e-10)
    b = 8
    Oms = [philox.gaussian(ph.shape[0], b, 70 + i).astype(np.float32).astype(np.float64) for i, ph in enumerate(phis)]
    U0 = batch.pack([torch.tensor(o, dtype=torch.float32, device="cuda") for o in Oms])
    for t in (1.0, 10.0):
        Y, _, _ = batch.expv(U0, [t, t], outer_dim=30)
        for i, (ph, om, y) in enumerate(zip(phis, Oms, batch.unpack(Y))):
            (ref,) = laplacian.expv(laplacian.walk_laplacian(ph), om, [t])
            err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)
            assert err < 1e-4, (t, i, err)


def test_batch_diffusion_on_disconnected_small_graphs(ctx, lib):
    """Small graphs with many components (lattices with edges kept w.p. 0.35 or 0.5:
    isolated nodes and small pieces) and one block with dependent columns: each graph's
    Krylov space stops growing by b per step as its components fill up, so the step at
    which the space is complete is not ceil(n / b).  exp(-t L) U0 against the dense
    oracle."""
    print("[gpu] batched diffusion on disconnected small graphs", flush=True)
    specs = [(9, 11, 0.35, 11), (12, 12, 0.5, 12), (8, 8, 0.35, 13), (10, 10, 0.9, 14)]
    graphs, descs, phis, Oms = [], [], [], []
    for i, (nx, ny, keep, seed) in enumerate(specs):
        rp, ci = synth.road_grid(nx, ny, keep, seed=seed)
        n = len(rp) - 1
        mu, kind = (1.0, "res") if i % 2 == 0 else (0.5, "exp")
        A = walks.adjacency(n, rp, ci)
        if kind == "exp":
            param = 1.0 / max(np.linalg.eigvalsh(A)[-1], 1e-12)
        else:
            param = 0.5 / max(walks.spectral_radius(walks.linearisation(A, mu)), 1e-3)
        graphs.append(lib.Graph(ctx, rp, ci, validate=True))
        descs.append({"mu": mu, "func": kind, "param": param})
        phis.append(genfun.phi(A, mu, kind, param))
        om = philox.gaussian(n, 8, 200 + i).astype(np.float32).astype(np.float64)
        if i == 3:
            om[:, 4:] = om[:, :4]  # dependent columns: rank 4
        Oms.append(om)
    batch = lib.Batch(ctx, graphs, descs, tol=1e-12)
    U0 = batch.pack([torch.tensor(o, dtype=torch.float32, device="cuda") for o in Oms])
    ts = [1.0, 0.5, 5.0, 2.0]
    Y, _, _ = batch.expv(U0, ts, outer_dim=30)
    for i, (ph, om, y, t) in enumerate(zip(phis, Oms, batch.unpack(Y), ts)):
        (ref,) = laplacian.expv(laplacian.walk_laplacian(ph), om, [t])
        err = np.linalg.norm(y.cpu().numpy().astype(np.float64) - ref) / np.linalg.norm(ref)
        print(f"[gpu]   graph {i} n={ph.shape[0]}: relative error {err:.2e}", flush=True)
        assert err < 1e-4, (i, err)
