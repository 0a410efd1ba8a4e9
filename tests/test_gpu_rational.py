"""Rational Krylov average return probability (Alg. 1) through the C ABI against the
oracle.

The library returns the poles it used; the oracle builds its (complex, exactly solved)
block rational Arnoldi basis from the same poles, so both estimate from the same space
and the same probes.  Differences come from the shifted solves (COCG to solve_tol), the
projection (Rayleigh quotient V^T L V against the reduced pencil, equal with exact
solves) and the vector precision.  Tolerances on p_hat: FP64 1e-7 relative (solves to
1e-12); FP32 2e-4 relative plus 1e-6 of the largest estimate (the basis is orthogonal
to ~1e-6, solves reach 1e-6, so a small p_hat at late t carries an absolute error of
that order); on e_hat, absolute in units of p_hat: FP64 1e-6, FP32 2e-3.  At t = 0, Y(0) = Omega / n exactly, so p_hat(0)
is the Nystrom estimate of the identity from Omega alone, to rounding at any size."""

import numpy as np
import pytest

import synth
from oracle import estimators, genfun, laplacian, rational, walks

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def dev(x, dtype):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def ba(n, m, seed):
    rp, ci = synth.barabasi_albert(n, m, seed)
    return rp, ci, walks.adjacency(n, rp, ci)


def compare(lib, op, Lap, Om, ts, t_max, dtype, rtol_p, atol_e, pole_time=1.0, solve_tol=1e-12):
    n = Lap.shape[0]
    rho = np.linalg.eigvalsh(Lap).max()
    p, e, poles, info = op.return_prob(dev(Om, dtype), ts, t_max, rho=rho, pole_time=pole_time,
                                       solve_tol=solve_tol, max_iters=2000)
    assert info["npoles"] == poles.size and info["rho"] == rho
    assert info["solve_res"] <= solve_tol
    po, eo, _ = rational.return_probability_estimate(Lap, Om, ts, t_max, rho, poles=poles)
    atol_p = 1e-6 * np.abs(po).max() if dtype == torch.float32 else 0.0
    np.testing.assert_allclose(p, po, rtol=rtol_p, atol=atol_p)
    np.testing.assert_allclose(e, eo, rtol=0, atol=atol_e * np.abs(po).max())
    tr0, te0, _, _ = estimators.xnys(Om, Om / n)
    if ts[0] == 0.0:
        assert abs(p[0] - tr0) < 1e-5 * abs(tr0) and abs(e[0] - te0) < 1e-5 * abs(tr0)
    return p, e, poles, info


@pytest.mark.parametrize("mu,pole_time", [(0.0, 1.0), (0.5, 1.0), (0.5, 10.0), (1.0, 1.0)])
def test_fp64_exponential(ctx, lib, mu, pole_time):
    print(f"[gpu] return_prob fp64 exp mu={mu} pole_time={pole_time}", flush=True)
    n = 300
    rp, ci, A = ba(n, 2, 17)
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, "exp", beta, dtype=torch.float64, tol=1e-15)
    Lap = laplacian.walk_laplacian(genfun.phi(A, mu, "exp", beta))
    Om = synth.gaussian_block(n, 4, seed=3)
    ts = [0.0, 0.1, 1.0, 5.0, 10.0]
    p, e, poles, info = compare(lib, op, Lap, Om, ts, 10.0, torch.float64, 1e-7, 1e-6, pole_time=pole_time)
    assert info["nblocks"] == 1 + poles.size
    # work: every COCG iteration a walk-Laplacian product (K series steps) on 2M columns,
    # plus the projection's products on the basis blocks
    K, M = op.info()[0], Om.shape[1]
    assert info["products"] == 2 * M * info["iters_total"] * K + info["nblocks"] * M * K


def test_fp64_resolvent_lanczos(ctx, lib):
    print("[gpu] return_prob fp64 res mu=1 lanczos", flush=True)
    n = 300
    rp, ci, A = ba(n, 3, 5)
    alpha = 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float64, krylov_dim=60, method="lanczos", tol=1e-14)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", alpha))
    Om = synth.gaussian_block(n, 5, seed=8)
    p, e, poles, info = compare(lib, op, Lap, Om, [0.0, 0.5, 2.0, 20.0], 20.0, torch.float64, 1e-7, 1e-6)
    # the resolvent's shifted solves take one sparse product per COCG iteration (plus
    # one for the solution); the projection K Lanczos steps per basis block
    K, M = op.info()[0], Om.shape[1]
    assert info["products"] == 2 * M * (info["iters_total"] + info["solves"]) + info["nblocks"] * M * K


def test_fp32_exponential_ba(ctx, lib):
    print("[gpu] return_prob fp32 BA n=1500", flush=True)
    n = 1500
    rp, ci, A = ba(n, 3, 11)
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.5, "exp", beta, dtype=torch.float32, tol=1e-9)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 0.5, "exp", beta))
    Om = synth.gaussian_block(n, 8, seed=21)
    compare(lib, op, Lap, Om, [0.0, 0.3, 3.0, 30.0], 30.0, torch.float32, 2e-4, 2e-3, solve_tol=1e-6)


@pytest.mark.parametrize("M", [5, 20])
def test_fp32_resolvent_column_groups(ctx, lib, M):
    """FP32 Lanczos operators run every product as 16-column groups (the blocks padded
    with zero columns): M = 5 pads to 16 (groups of 2 and 1), M = 20 to 32 (4 and 2)."""
    print(f"[gpu] return_prob fp32 res mu=1 column groups M={M}", flush=True)
    n = 2500
    rp, ci, A = ba(n, 3, 23)
    alpha = 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float32, krylov_dim=30, method="lanczos", tol=1e-7)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", alpha))
    Om = synth.gaussian_block(n, M, seed=31)
    compare(lib, op, Lap, Om, [0.0, 0.5, 5.0, 50.0], 50.0, torch.float32, 2e-4, 2e-3, solve_tol=1e-6)


def test_fp32_resolvent_road_one_pass(ctx, lib):
    """A road-like lattice (every degree at most 4) with M = 30 probes (padded to 32
    columns) at alpha = 1 / (1 + rho(Z_1)): the shifted solves take the one-pass product
    (gather, shift and p^T q in one kernel), as on the road-network workload."""
    print("[gpu] return_prob fp32 res mu=1 road lattice, one-pass solve product", flush=True)
    rp, ci = synth.road_grid(50, 50, 0.7, seed=3)
    n = len(rp) - 1
    A = walks.adjacency(n, rp, ci)
    assert np.diff(rp).max() <= 4
    alpha = 1.0 / (1.0 + walks.spectral_radius(walks.linearisation(A, 1.0)))
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float32, krylov_dim=30, method="lanczos", tol=1e-7)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", alpha))
    Om = synth.gaussian_block(n, 30, seed=41)
    compare(lib, op, Lap, Om, [0.0, 0.5, 5.0, 50.0], 50.0, torch.float32, 2e-4, 2e-3, solve_tol=1e-6)


@pytest.mark.parametrize("nx,ny,keep,M", [(9, 11, 0.7, 4), (9, 11, 0.35, 4), (12, 12, 0.5, 6)])
def test_fp32_resolvent_small_one_pass(ctx, lib, nx, ny, keep, M):
    """The one-pass solve product on small lattices: fewer rows than the grid's row groups,
    some XCD row ranges short or empty, isolated nodes (keep 0.35 and 0.5), against the
    oracle from the library's poles.  The basis (10 blocks of M) stays below n, where the
    oracle's basis (no deflation) is well defined.  The blocks are padded to 16 columns,
    so the projection's Lanczos runs start from rank-deficient blocks: this case found
    that the step count was capped for full-rank blocks (n / 16 + 1 steps, 8 here)."""
    print(f"[gpu] return_prob fp32 res one-pass product, lattice {nx}x{ny} keep {keep} M={M}", flush=True)
    rp, ci = synth.road_grid(nx, ny, keep, seed=11)
    n = len(rp) - 1
    A = walks.adjacency(n, rp, ci)
    alpha = 0.5 / max(walks.spectral_radius(walks.linearisation(A, 1.0)), 1e-3)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float32, krylov_dim=30, method="lanczos", tol=1e-7)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", alpha))
    Om = synth.gaussian_block(n, M, seed=5)
    _, _, _, info = compare(lib, op, Lap, Om, [0.0, 0.5, 5.0], 5.0, torch.float32, 2e-4, 2e-3, solve_tol=1e-6)
    assert info["nblocks"] * M < n


@pytest.mark.parametrize("M", [8, 30])
def test_fp32_resolvent_long_rows(ctx, lib, M):
    """A node joined to 400 others (above the one-pass product's row limit of 256): the
    shifted solves take the sparse-product kernel and the separate shift pass."""
    print(f"[gpu] return_prob fp32 res mu=1 with a long row, M={M}", flush=True)
    n = 2000
    rp, ci = synth.barabasi_albert(n, 3, 29)
    rows = np.repeat(np.arange(n), np.diff(rp))
    extra = np.random.default_rng(5).choice(np.arange(1, n), 400, replace=False)
    rp, ci = synth.csr_from_edges(n, np.concatenate([rows, np.zeros(400, dtype=np.int64)]),
                                  np.concatenate([ci, extra]))
    assert np.diff(rp).max() > 256
    A = walks.adjacency(n, rp, ci)
    alpha = 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 1.0, "res", alpha, dtype=torch.float32, krylov_dim=30, method="lanczos", tol=1e-7)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 1.0, "res", alpha))
    Om = synth.gaussian_block(n, M, seed=43)
    compare(lib, op, Lap, Om, [0.0, 0.5, 5.0, 50.0], 50.0, torch.float32, 2e-4, 2e-3, solve_tol=1e-6)


def test_buffers_kept_between_calls(ctx, lib):
    """The work buffers and the column-group runners stay with the operator between
    calls: calls of different widths in a row on one operator (Mp = 32, 16, 32, 16)
    give what a fresh operator gives, bit for bit."""
    print("[gpu] return_prob buffers kept between calls", flush=True)
    n = 1500
    rp, ci, A = ba(n, 3, 17)
    alpha = 0.5 / walks.spectral_radius(walks.linearisation(A, 1.0))
    g = lib.Graph(ctx, rp, ci)

    def make():
        return lib.Operator(g, 1.0, "res", alpha, dtype=torch.float32, krylov_dim=30, method="lanczos", tol=1e-7)

    ts = [0.0, 0.5, 5.0]
    op = make()
    for M in (20, 5, 24, 8):
        Om = dev(synth.gaussian_block(n, M, seed=M), torch.float32)
        p1, e1, _, i1 = op.return_prob(Om, ts, 10.0, rho=0.0, solve_tol=1e-6, max_iters=2000)
        fresh = make()
        p2, e2, _, i2 = fresh.return_prob(Om, ts, 10.0, rho=0.0, solve_tol=1e-6, max_iters=2000)
        fresh.close()
        assert i1["iters_total"] == i2["iters_total"]
        np.testing.assert_array_equal(p1, p2)
        np.testing.assert_array_equal(e1, e2)
    op.close()


def test_estimated_rho_and_components_limit(ctx, lib):
    print("[gpu] return_prob components limit, estimated rho", flush=True)
    blocks = []
    for seed in (1, 2, 3):
        rp, ci, A = ba(60, 2, seed)
        blocks.append(A)
    import scipy.linalg as sla
    A = sla.block_diag(*blocks)
    n = A.shape[0]
    rp, ci = synth.csr_from_dense(A)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.0, "exp", 0.2, dtype=torch.float64, tol=1e-15)
    Lap = laplacian.walk_laplacian(genfun.phi(A, 0.0, "exp", 0.2))
    lam = np.sort(np.linalg.eigvalsh(Lap))
    t_end = 200.0 / lam[3]
    Om = synth.gaussian_block(n, 6, seed=4)
    p, e, poles, info = op.return_prob(dev(Om, torch.float64), [0.0, t_end], t_end, rho=0.0, pole_time=t_end,
                                       solve_tol=1e-12, max_iters=4000)
    assert lam[-1] * (1 - 1e-9) <= info["rho"] <= 1.05 * lam[-1], (info["rho"], lam[-1])
    assert abs(p[1] - 3.0 / n) < 1e-8 and e[1] < 1e-8


def test_rank_deficient_probes(ctx, lib):
    print("[gpu] return_prob rank-deficient probe block", flush=True)
    n = 200
    rp, ci, A = ba(n, 2, 9)
    beta = 1.0 / np.linalg.eigvalsh(A)[-1]
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.0, "exp", beta, dtype=torch.float64, tol=1e-15)
    Om = synth.gaussian_block(n, 4, seed=2)
    Om[:, 3] = Om[:, 1]
    p, e, poles, info = op.return_prob(dev(Om, torch.float64), [0.0, 1.0, 4.0], 4.0, solve_tol=1e-10)
    assert np.all(np.isfinite(p)) and np.all(np.isfinite(e))
    tr0, te0, _, _ = estimators.xnys(Om, Om / n)
    assert abs(p[0] - tr0) < 1e-8 * abs(tr0)


def test_bad_arguments(ctx, lib):
    print("[gpu] return_prob bad arguments", flush=True)
    n = 100
    rp, ci, A = ba(n, 2, 1)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.0, "exp", 0.1, dtype=torch.float64, tol=1e-12)
    Om = dev(synth.gaussian_block(n, 4, seed=1), torch.float64)
    with pytest.raises(lib.WLError):
        op.return_prob(dev(synth.gaussian_block(n, 1, seed=1), torch.float64), [1.0], 1.0)
    with pytest.raises(lib.WLError):
        op.return_prob(dev(synth.gaussian_block(n, 33, seed=1), torch.float64), [1.0], 1.0)
    with pytest.raises(lib.WLError):
        op.return_prob(Om, [-1.0], 1.0)
    with pytest.raises(lib.WLError):
        op.return_prob(Om, [1.0], 0.0)
    with pytest.raises(lib.WLError):
        op.return_prob(Om, [1.0], 1.0, pole_time=0.0)
    with pytest.raises(lib.WLError):
        op.return_prob(Om, [1.0], 1.0, solve_tol=0.0)
    # an unreachable iteration budget is reported, not hidden
    with pytest.raises(lib.WLError):
        op.return_prob(Om, [1.0], 1.0, solve_tol=1e-14, max_iters=1)


def test_edgeless_graph(ctx, lib):
    """No edges: L = 0, rho(L) = 0, no poles; exp(-t L) = I, so every p_hat(t) is the
    Nystrom estimate of I / n from the probes."""
    print("[gpu] return_prob edgeless graph", flush=True)
    n = 40
    g = lib.Graph(ctx, np.zeros(n + 1, dtype=np.int32), np.zeros(0, dtype=np.int32), validate=True)
    Om = synth.gaussian_block(n, 5, seed=7)
    tr0, te0, _, _ = estimators.xnys(Om, Om / n)
    for kind in ("exp", "res"):
        op = lib.Operator(g, 0.5, kind, 0.3, dtype=torch.float64, krylov_dim=5)
        p, e, poles, info = op.return_prob(dev(Om, torch.float64), [0.0, 1.0, 50.0], 50.0, rho=0.0)
        assert poles.size == 0 and info["nblocks"] == 1 and info["rho"] < 1e-12
        np.testing.assert_allclose(p, tr0, rtol=1e-10)
        np.testing.assert_allclose(e, te0, rtol=1e-8, atol=1e-14)


def test_standard_laplacian(ctx, lib):
    """Linear weights f(x) = x give phi = I + A and L = D - A, the standard Laplacian
    Alg. 1 also takes (the paper's reference Laplacian in its return-probability
    figures)."""
    print("[gpu] return_prob standard Laplacian", flush=True)
    n = 300
    rp, ci, A = ba(n, 2, 19)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.0, "linear", 1.0, dtype=torch.float64)
    assert op.info() == (1, lib.WL_M_RECURRENCE)
    d = A.sum(1)
    X = synth.gaussian_block(n, 3, seed=4)
    np.testing.assert_allclose(host(op.fdeg()), 1.0 + d, rtol=1e-14)
    Lap = np.diag(d) - A
    np.testing.assert_allclose(host(op.apply_L(dev(X, torch.float64))), Lap @ X, atol=1e-12)
    Om = synth.gaussian_block(n, 4, seed=5)
    compare(lib, op, Lap, Om, [0.0, 0.2, 2.0, 20.0], 20.0, torch.float64, 1e-7, 1e-6)
    with pytest.raises(lib.WLError):
        lib.Operator(g, 0.0, "linear", 1.0, dtype=torch.float64, method="lanczos")


@pytest.mark.parametrize("mu,kind,dtype", [(0.5, "exp", "f64"), (1.0, "res", "f64"), (0.5, "exp", "f32"),
                                          (1.0, "res", "f32")])
def test_pole_independent_estimates(ctx, lib, mu, kind, dtype):
    """Each side builds its own AAA poles (the library on the device path, the oracle
    with LAPACK), so the check does not depend on the library's poles:
      * each p_hat(t) lies within 5 e_hat(t) of the exact tr exp(-t L) / n (Alg. 1
        returns the estimate with its error estimate);
      * the two estimates agree with each other: both spaces reproduce exp(-t L) Omega
        to ~1e-10 on these graphs (measured with the oracle against the exact
        exp(-t L) Omega), so the bound is that of the shifted solves and the vector
        precision: FP64 1e-8 relative, FP32 2e-4 relative plus 1e-6 of the largest."""
    print(f"[gpu] return_prob pole-independent mu={mu} {kind} {dtype}", flush=True)
    n = 400
    rp, ci, A = ba(n, 3, 5)
    if kind == "exp":
        param = 1.0 / np.linalg.eigvalsh(A)[-1]
        method, kd = "auto", 0
    else:
        param = 1.0 / (1.0 + walks.spectral_radius(walks.linearisation(A, mu)))
        method, kd = "lanczos", 60
    td = torch.float64 if dtype == "f64" else torch.float32
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, kind, param, dtype=td, krylov_dim=kd, method=method,
                      tol=1e-15 if dtype == "f64" else 1e-9)
    Lap = laplacian.walk_laplacian(genfun.phi(A, mu, kind, param))
    Om = synth.gaussian_block(n, 8, seed=3)
    ts = [0.0, 0.1, 1.0, 5.0, 10.0]
    rho = np.linalg.eigvalsh(Lap).max()
    solve_tol = 1e-12 if dtype == "f64" else 1e-6
    p, e, poles_lib, info = op.return_prob(dev(Om, td), ts, 10.0, rho=rho, solve_tol=solve_tol, max_iters=2000)
    po, eo, poles_orc = rational.return_probability_estimate(Lap, Om, ts, 10.0, rho)
    exact = rational.exact_return_probability(Lap, ts)
    print(f"[gpu] poles: library {poles_lib.size}, oracle {poles_orc.size}; "
          f"|p - exact| / e_hat: {np.round(np.abs(p - exact) / e, 2)}", flush=True)
    # where e_hat vanishes (at late t exp(-t L) Omega is nearly the rank-one projection
    # on the constant vector, which Nystrom recovers exactly) the FP32 estimate keeps
    # its rounding: 1e-6 of the largest estimate, as in the parity tests above
    floor = 1e-6 * np.abs(po).max() if dtype == "f32" else 1e-10 * np.abs(po).max()
    assert np.all(np.abs(p - exact) <= 5 * e + floor) and np.all(np.abs(po - exact) <= 5 * eo + 1e-12)
    if dtype == "f64":
        np.testing.assert_allclose(p, po, rtol=1e-8, atol=0)
    else:
        np.testing.assert_allclose(p, po, rtol=2e-4, atol=1e-6 * np.abs(po).max())


@pytest.mark.parametrize("mu,frac", [(1.0, 0.5), (0.0, 0.3)])
def test_resolvent_rho_bound(ctx, lib, mu, frac):
    """Without a caller's rho, a resolvent takes the bound max w - s / (s + (mu alpha^2 +
    alpha) d_max): phi = s A_mu^{-1} is positive definite, so L <= diag(w), and
    lambda_max(A_mu) is bounded by its largest Gershgorin row.  It must lie above
    lambda_max(L) (and within 50% of it on these graphs: 13% and 31% above, measured with
    the oracle; 3% on the road stand-in of the bench),
    cost no sparse product, and the estimate on the wider interval must still match the
    exact tr exp(-t L) / n within its error estimate."""
    print(f"[gpu] return_prob resolvent rho bound mu={mu}", flush=True)
    n = 300
    rp, ci, A = ba(n, 3, 5)
    rz = walks.spectral_radius(walks.linearisation(A, mu)) if mu > 0 else np.linalg.eigvalsh(A)[-1]
    alpha = frac / rz
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, mu, "res", alpha, dtype=torch.float64, krylov_dim=60, method="lanczos", tol=1e-14)
    Lap = laplacian.walk_laplacian(genfun.phi(A, mu, "res", alpha))
    lmax = np.linalg.eigvalsh(Lap).max()
    Om = synth.gaussian_block(n, 6, seed=12)
    ts = [0.0, 0.5, 2.0, 10.0]
    p, e, poles, info = op.return_prob(dev(Om, torch.float64), ts, 10.0, rho=0.0, solve_tol=1e-12, max_iters=2000)
    assert lmax * (1 - 1e-9) <= info["rho"] <= 1.5 * lmax, (info["rho"], lmax)
    K, M = op.info()[0], Om.shape[1]
    assert info["products"] == 2 * M * (info["iters_total"] + info["solves"]) + info["nblocks"] * M * K
    exact = rational.exact_return_probability(Lap, ts)
    assert np.all(np.abs(p - exact) <= 5 * e + 1e-10 * np.abs(exact).max()), (p, exact, e)
