"""wl_apply_L_noalloc (the walk-Laplacian product on the library's fixed device region,
for callers that cannot allocate) through the C ABI: the same results as wl_apply_L on
two calls in a row, the second with a smaller input, no device allocation inside the
calls, and the size limit of the region."""

import numpy as np
import pytest

import synth
from oracle import sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

REGION = 64 << 20


def _graph(n, seed):
    rp, ci = synth.barabasi_albert(n, 5, seed)
    return n, rp, ci, sparse.adjacency(n, rp, ci)


CASES = [
    ("exp", 0.5, torch.float32, "auto"),
    ("res", 0.5, torch.float64, "auto"),
    ("res", 0.25, torch.float32, "lanczos"),
]


@pytest.mark.parametrize("kind,mu,dtype,method", CASES)
def test_noalloc_equals_apply_L(lib, kind, mu, dtype, method):
    print(f"[gpu] noalloc {kind} mu={mu} {dtype} {method}", flush=True)
    ctx = lib.Context(0)
    runs = []
    for n, seed, b in ((8000, 11, 16), (3000, 12, 4)):  # second call: smaller graph and block
        n, rp, ci, As = _graph(n, seed)
        g = lib.Graph(ctx, rp, ci)
        lam = sparse.lambda_max(As)
        param = 1.0 / lam if kind == "exp" else 0.5 / sparse.rho_Z(As, mu)
        op = lib.Operator(g, mu, kind, param, dtype=dtype, krylov_dim=30, method=method)
        X = torch.tensor(synth.rademacher_block(n, b, 3), dtype=dtype, device="cuda")
        ref = lib.Operator(g, mu, kind, param, dtype=dtype, krylov_dim=30, method=method).apply_L(X)
        assert op.workspace_size("apply_L", b) <= REGION
        out = torch.empty_like(X)
        runs.append((op, X, out, ref))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for op, X, out, ref in runs:
        op.apply_L_noalloc(X, out)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (2 << 20), (free0, free1)
    for op, X, out, ref in runs:
        # same kernels in the same order on other buffers: bit for bit
        assert torch.equal(out, ref), float((out - ref).abs().max())
    # once the walk degrees are cached, repeated calls still agree
    op, X, out, ref = runs[0]
    op.fdeg()
    out.zero_()
    op.apply_L_noalloc(X, out)
    assert torch.equal(out, ref)


def test_noalloc_region_limit(lib):
    print("[gpu] noalloc region limit", flush=True)
    ctx = lib.Context(0)
    n, rp, ci, As = _graph(20000, 11)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.5, "res", 0.5 / sparse.rho_Z(As, 0.5), dtype=torch.float64, krylov_dim=30,
                      method="lanczos")
    b = 64
    assert op.workspace_size("apply_L", b) > REGION
    X = torch.tensor(synth.rademacher_block(n, b, 3), dtype=torch.float64, device="cuda")
    out = torch.full_like(X, 7.0)
    with pytest.raises(lib.WLError, match="ERANGE"):
        op.apply_L_noalloc(X, out)
    assert bool((out == 7.0).all())  # nothing was enqueued
    # the operator still works on the allocating path afterwards
    Y = op.apply_L(X[:, :8].contiguous())
    ref = sparse.phi_res_apply(As, 0.5, 0.5 / sparse.rho_Z(As, 0.5), X[:, :8].cpu().numpy())
    assert np.isfinite(Y.cpu().numpy()).all() and np.isfinite(ref).all()
