"""Walk degrees evaluated beside the blocks (wl_multi_apply_fdeg): the vectors of ones
of every operator ride in one extra 16-column group of the wide block, so one sparse
product per step serves phi_g X (or L_g X) and w_g = phi_g 1 of all operators.
Compared with the separate calls (wl_multi_apply, wl_multi_fdeg) and with the oracle.
Series: FP64 1e-12 / 1e-8 (only the summation order differs), FP32 1e-6 / 2e-5.
Lanczos (FP32, 16-column groups; the ones' group holds independent single-column
processes with diagonal Grams): 2e-5 against the separate calls and the oracle, the
walk degrees also node by node (largest relative error over all nodes 1e-5)."""

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


@pytest.fixture(scope="module")
def ba20k(ctx, lib):
    n = 20000
    rp, ci = synth.barabasi_albert(n, 5, 11)
    As = sparse.adjacency(n, rp, ci)
    g = lib.Graph(ctx, rp, ci)
    return n, As, g, g.lambda_max()


def test_series_fp64_packed_equals_separate(ctx, lib):
    print("[gpu] multi fdeg series fp64", flush=True)
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    specs = [(0.0, "exp", 1.0 / lam, 0), (0.5, "res", 0.5 / lam, 45), (1.0, "exp", 1.0 / lam, 0),
             (0.25, "exp", 0.5 / lam, 0)]
    ops = [lib.Operator(g, mu, f, p, dtype=torch.float64, krylov_dim=K, method="recurrence")
           for mu, f, p, K in specs]
    multi = lib.Multi(ops)
    for b in (3, 4):  # scalar and vector epilogues
        X = synth.gaussian_block(n, b, 5)
        Xd = dev(X, torch.float64)
        for lap in (True, False):
            Y, W = multi.apply_fdeg(Xd, laplacian=lap)
            Y, W = host(Y), host(W)
            Ys = host(multi.apply_L(Xd) if lap else multi.apply_phi(Xd))
            Ws = host(multi.fdeg())
            assert np.linalg.norm(W - Ws) <= 1e-12 * np.linalg.norm(Ws), (b, lap)
            assert np.linalg.norm(Y - Ys) <= 1e-12 * np.linalg.norm(Ys), (b, lap)
            for i, (mu, f, p, K) in enumerate(specs):
                ph = genfun.phi(A, mu, f, p)
                w = ph.sum(1)
                assert np.linalg.norm(W[:, i] - w) < 1e-8 * np.linalg.norm(w)
                ref = laplacian.apply_laplacian(ph, X) if lap else ph @ X
                scale = np.linalg.norm(w[:, None] * X) + np.linalg.norm(ph @ X)
                assert np.linalg.norm(Y[:, i * b:(i + 1) * b] - ref) < 1e-8 * scale, (b, lap, i)


@pytest.mark.parametrize("kind", ["exp", "res"])
def test_fp32_five_operators_block16(ba20k, lib, kind):
    """The default workload's shape: five operators x 16 columns plus the ones' group,
    96 FP32 values per row (three whole cache lines)."""
    n, As, g, lam = ba20k
    print(f"[gpu] multi fdeg fp32 {kind} BA20k", flush=True)
    mus = [0.0, 0.25, 0.5, 0.75, 1.0]
    params = [1.0 / lam if kind == "exp" else 0.5 / sparse.rho_Z(As, mu) for mu in mus]
    ops = [lib.Operator(g, mu, kind, p, dtype=torch.float32, krylov_dim=30) for mu, p in zip(mus, params)]
    multi = lib.Multi(ops)
    X = synth.rademacher_block(n, 16, 3)
    Xd = dev(X, torch.float32)
    Y, W = multi.apply_fdeg(Xd)
    Y, W = host(Y), host(W)
    Ys, Ws = host(multi.apply_L(Xd)), host(multi.fdeg())
    sep = 1e-6 if kind == "exp" else 2e-5
    for i, (mu, p) in enumerate(zip(mus, params)):
        cols = slice(16 * i, 16 * (i + 1))
        wr = sparse.fdeg(As, mu, kind, p)
        pr = sparse.phi_apply(As, mu, kind, p, X)
        scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(pr)
        assert np.linalg.norm(Y[:, cols] - Ys[:, cols]) < sep * scale, (mu, "vs separate")
        assert np.linalg.norm(Y[:, cols] - (wr[:, None] * X - pr)) < 2e-5 * scale, (mu, "vs oracle")
        assert np.linalg.norm(W[:, i] - Ws[:, i]) < sep * np.linalg.norm(wr), (mu, "w vs separate")
        assert np.linalg.norm(W[:, i] - wr) < 1e-5 * np.linalg.norm(wr), (mu, "w vs oracle")
        worst = float(np.max(np.abs(W[:, i] - wr) / np.abs(wr)))
        assert worst < 1e-5, (mu, worst)  # node by node (hubs do not hide the leaves)
    # repeated calls give the same result (buffers reused, nothing left over)
    Y2, W2 = multi.apply_fdeg(Xd)
    assert np.array_equal(host(Y2), Y) and np.array_equal(host(W2), W)


def test_lanczos_phi_and_single_operator(ba20k, lib):
    """apply_phi form and one operator (nops = 1: the ones' group holds one column)."""
    n, As, g, lam = ba20k
    print("[gpu] multi fdeg lanczos phi nops=1", flush=True)
    mu = 0.5
    p = 0.5 / sparse.rho_Z(As, mu)
    op = lib.Operator(g, mu, "res", p, dtype=torch.float32, krylov_dim=30)
    multi = lib.Multi([op])
    X = synth.gaussian_block(n, 16, 7)
    Xd = dev(X, torch.float32)
    Y, W = multi.apply_fdeg(Xd, laplacian=False)
    wr = sparse.fdeg(As, mu, "res", p)
    pr = sparse.phi_apply(As, mu, "res", p, X)
    assert np.linalg.norm(host(Y) - pr) < 2e-5 * np.linalg.norm(pr)
    assert np.linalg.norm(host(W)[:, 0] - wr) < 1e-5 * np.linalg.norm(wr)


def test_uncovered_shapes_fall_back(ctx, lib):
    """FP64 Lanczos operators (no grouped kernels for the packed block): the separate
    calls, one after the other, with identical results."""
    print("[gpu] multi fdeg fallback", flush=True)
    n = 400
    rp, ci = synth.erdos_renyi_gnm(n, 1600, 21)
    A = walks.adjacency(n, rp, ci)
    lam = np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    ops = [lib.Operator(g, mu, "res", 0.5 / lam, dtype=torch.float64, krylov_dim=40, method="lanczos")
           for mu in (0.0, 0.5)]
    multi = lib.Multi(ops)
    X = synth.gaussian_block(n, 16, 5)
    Xd = dev(X, torch.float64)
    Y, W = multi.apply_fdeg(Xd)
    assert torch.equal(Y, multi.apply_L(Xd)) and torch.equal(W, multi.fdeg())


def test_argument_checks(ba20k, lib):
    n, As, g, lam = ba20k
    op = lib.Operator(g, 0.5, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=10)
    multi = lib.Multi([op])
    X = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(lib.WLError, match="EINVAL"):
        lib._lib.check(lib.load().wl_multi_apply_fdeg(multi.handle, lib._ptr(X), 16, 1, lib._ptr(Y), lib._ptr(Y), 1))
    with pytest.raises(lib.WLError, match="EINVAL"):
        lib._lib.check(lib.load().wl_multi_apply_fdeg(multi.handle, lib._ptr(X), 16, 2, lib._ptr(Y), lib._ptr(X), 1))


@pytest.mark.parametrize("kind", ["exp", "res"])
def test_fewer_blocks_than_walk_degrees(ba20k, lib, kind):
    """nx < nops: L_g X for the first nx operators, walk degrees of all of them (the
    resolvent layout of the default workload: one operator's block beside all five
    walk-degree processes, 32 FP32 values per row)."""
    n, As, g, lam = ba20k
    print(f"[gpu] multi fdeg nx<nops {kind}", flush=True)
    mus = [1.0, 0.0, 0.25, 0.5, 0.75]
    params = [1.0 / lam if kind == "exp" else 0.5 / sparse.rho_Z(As, mu) for mu in mus]
    ops = [lib.Operator(g, mu, kind, p, dtype=torch.float32, krylov_dim=30) for mu, p in zip(mus, params)]
    multi = lib.Multi(ops)
    X = synth.rademacher_block(n, 16, 4)
    Xd = dev(X, torch.float32)
    for nx in (1, 2):
        Y, W = multi.apply_fdeg(Xd, nx=nx)
        Y, W = host(Y), host(W)
        assert Y.shape == (n, 16 * nx) and W.shape == (n, 5)
        for i, (mu, p) in enumerate(zip(mus, params)):
            wr = sparse.fdeg(As, mu, kind, p)
            assert np.linalg.norm(W[:, i] - wr) < 1e-5 * np.linalg.norm(wr), (nx, mu)
            assert float(np.max(np.abs(W[:, i] - wr) / np.abs(wr))) < 1e-5, (nx, mu)
            if i < nx:
                pr = sparse.phi_apply(As, mu, kind, p, X)
                scale = np.linalg.norm(wr[:, None] * X) + np.linalg.norm(pr)
                single = host(ops[i].apply_L(Xd))
                assert np.linalg.norm(Y[:, 16 * i:16 * (i + 1)] - (wr[:, None] * X - pr)) < 2e-5 * scale, (nx, mu)
                assert np.linalg.norm(Y[:, 16 * i:16 * (i + 1)] - single) < 2e-5 * scale, (nx, mu)
