"""Failure handling through the C ABI, every condition forced from the host:

* injected allocation failures (wl_test_fail_alloc, WL_TEST_FAIL_ALLOC): the k-th device
  allocation of a call fails as an out-of-memory would; the call returns WL_ENOMEM and
  the same handles then give the result of an undisturbed call;
* the output scan (wl_ctx_set_checks(WL_CHECK_FINITE)): NaN or Inf in an output becomes
  WL_ENUMERIC, clean outputs pass unchanged;
* trace mode (WL_TRACE): destroying the context prints every timed kernel class."""

import os
import subprocess
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


@pytest.fixture(scope="module")
def ba(ctx, lib):
    n = 3000
    rp, ci = synth.barabasi_albert(n, 5, 3)
    return n, rp, ci, lib.Graph(ctx, rp, ci)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def run_with_failures(lib, make, call, ref, rtol, kmax=64):
    """For k = 0, 1, ...: a fresh handle from make(), the k-th allocation of call(h)
    made to fail; every failing call must raise WL_ENOMEM and the same handle must then
    return ref.  Stops at the first k the call does not reach.  Returns the number of
    failures seen."""
    fails = 0
    try:
        for k in range(kmax):
            h = make()
            lib.inject_alloc_failure(k)
            try:
                out = call(h)
                lib.inject_alloc_failure(-1)
                np.testing.assert_allclose(out, ref, rtol=rtol, atol=rtol * np.abs(ref).max())
                return fails
            except lib.WLError as e:
                lib.inject_alloc_failure(-1)
                assert "NOMEM" in str(e) and "injected" in str(e), (k, str(e))
                fails += 1
            out = call(h)  # the same handle after the failure
            np.testing.assert_allclose(out, ref, rtol=rtol, atol=rtol * np.abs(ref).max())
        raise AssertionError(f"the call still allocated after {kmax} injected failures")
    finally:
        lib.inject_alloc_failure(-1)


def test_injected_failures_apply_L(ctx, lib, ba):
    print("[gpu] injected allocation failures: apply_L, FP32 Lanczos resolvent", flush=True)
    n, rp, ci, g = ba
    X = torch.tensor(synth.gaussian_block(n, 16, 5), dtype=torch.float32, device="cuda")

    def make():
        return lib.Operator(g, 0.5, "res", 0.3 / g.spectral_radius(0.5), dtype=torch.float32, method="lanczos")

    ref = host(make().apply_L(X))
    fails = run_with_failures(lib, make, lambda op: host(op.apply_L(X)), ref, 1e-6)
    print(f"[gpu]   {fails} allocations failed in turn", flush=True)
    assert fails >= 2


def test_injected_failures_expv(ctx, lib, ba):
    print("[gpu] injected allocation failures: expv, FP64 series", flush=True)
    n, rp, ci, g = ba
    U0 = torch.tensor(synth.spike_block(n, [0, 7, 99, 1500]), dtype=torch.float64, device="cuda")

    def make():
        return lib.Operator(g, 0.25, "exp", 0.05, dtype=torch.float64)

    def call(op):
        (y1, y2), _ = op.expv(U0, [0.5, 2.0], outer_dim=12)
        return np.concatenate([host(y1), host(y2)])

    ref = call(make())
    fails = run_with_failures(lib, make, call, ref, 1e-12)
    print(f"[gpu]   {fails} allocations failed in turn", flush=True)
    assert fails >= 2


def test_injected_failures_return_prob(ctx, lib):
    print("[gpu] injected allocation failures: return_prob, FP32 resolvent", flush=True)
    n = 1500
    rp, ci = synth.barabasi_albert(n, 3, 11)
    g = lib.Graph(ctx, rp, ci)
    Om = torch.tensor(synth.gaussian_block(n, 5, 2), dtype=torch.float32, device="cuda")
    rho = g.spectral_radius(1.0)

    def make():
        return lib.Operator(g, 1.0, "res", 0.5 / rho, dtype=torch.float32, method="lanczos", krylov_dim=30)

    def call(op):
        p, e, poles, info = op.return_prob(Om, [0.5, 5.0], 5.0, rho=4.0, solve_tol=1e-6)
        return np.asarray(p)

    ref = call(make())
    fails = run_with_failures(lib, make, call, ref, 1e-6)
    print(f"[gpu]   {fails} allocations failed in turn", flush=True)
    assert fails >= 2


def test_injected_failure_graph_create(ctx, lib):
    print("[gpu] injected allocation failure: graph creation", flush=True)
    n = 500
    rp, ci = synth.barabasi_albert(n, 3, 2)
    lib.inject_alloc_failure(0)
    try:
        with pytest.raises(lib.WLError, match="NOMEM"):
            lib.Graph(ctx, rp, ci, copy=True)
    finally:
        lib.inject_alloc_failure(-1)
    g = lib.Graph(ctx, rp, ci, copy=True, validate=True)
    assert g.n == n


def test_injected_failure_from_environment(lib):
    """WL_TEST_FAIL_ALLOC=0 in a fresh process: its first library allocation (the graph's
    hub-row list) fails; the next graph is made."""
    print("[gpu] injected allocation failure from the environment", flush=True)
    code = (
        "import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import torch, synth, paper_2601_11338_amd as wl\n"
        "rp, ci = synth.barabasi_albert(400, 3, 1)\n"
        "ctx = wl.Context(0)\n"
        "try:\n"
        "    wl.Graph(ctx, rp, ci)\n"
        "    print('no failure')\n"
        "except wl.WLError as e:\n"
        "    print('failed:', e)\n"
        "g = wl.Graph(ctx, rp, ci)\n"
        "print('second graph', g.n)\n" % (ROOT, os.path.join(ROOT, "tests")))
    env = dict(os.environ, WL_TEST_FAIL_ALLOC="0")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "failed:" in r.stdout and "NOMEM" in r.stdout and "second graph 400" in r.stdout, r.stdout


def test_output_scan(ctx, lib, ba):
    print("[gpu] NaN / Inf scan of outputs", flush=True)
    n, rp, ci, g = ba
    op = lib.Operator(g, 0.5, "exp", 0.05, dtype=torch.float32)
    X = torch.tensor(synth.gaussian_block(n, 8, 9), dtype=torch.float32, device="cuda")
    Xbad = X.clone()
    Xbad[17, 3] = float("nan")
    Xinf = X.clone()
    Xinf[2000, 0] = float("inf")
    clean = host(op.apply_L(X))
    assert not np.all(np.isfinite(host(op.apply_L(Xbad))))  # checks off: the NaN goes through
    ctx.set_checks(True)
    try:
        np.testing.assert_array_equal(host(op.apply_L(X)), clean)
        np.testing.assert_array_equal(host(op.fdeg()), host(op.fdeg()))
        for bad in (Xbad, Xinf):
            with pytest.raises(lib.WLError, match="NUMERIC|NaN or Inf"):
                op.apply_L(bad)
            with pytest.raises(lib.WLError, match="NUMERIC|NaN or Inf"):
                op.apply_phi(bad)
        U0 = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
        U0[5, 0] = U0[9, 1] = 1.0
        op.expv(U0, [1.0], outer_dim=8)
        U0[11, 1] = float("nan")
        with pytest.raises(lib.WLError, match="NUMERIC|NaN or Inf|non-finite"):
            op.expv(U0, [1.0], outer_dim=8)
    finally:
        ctx.set_checks(False)
    assert not np.all(np.isfinite(host(op.apply_L(Xbad))))


def test_trace_mode(lib, capfd):
    print("[gpu] trace mode", flush=True)
    n = 2000
    rp, ci = synth.barabasi_albert(n, 4, 6)
    os.environ["WL_TRACE"] = "1"
    try:
        c = lib.Context(0)
    finally:
        del os.environ["WL_TRACE"]
    g = lib.Graph(c, rp, ci)
    op = lib.Operator(g, 0.0, "exp", 0.1, dtype=torch.float32)
    X = torch.tensor(synth.gaussian_block(n, 16, 1), dtype=torch.float32, device="cuda")
    for _ in range(3):
        op.apply_L(X)
    op.close()
    g.close()
    c.close()
    err = capfd.readouterr().err
    assert "[walklap trace]" in err and "recurrence step" in err, err[-2000:]
