"""Caller-provided workspace (wl_workspace_size and the _ws variants): the same
results as the library-allocated calls, bit for bit (the same kernels in the same order
on other buffers), no device allocation inside the call, and argument checks."""

import ctypes as C

import numpy as np
import pytest

import synth
from oracle import sparse

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ba20k():
    n = 20000
    rp, ci = synth.barabasi_albert(n, 5, 11)
    return n, rp, ci, sparse.adjacency(n, rp, ci)


def work_for(op, call, b, outer_dim=0):
    nbytes = op.workspace_size(call, b, outer_dim)
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda"), nbytes


CASES = [
    ("exp", 0.5, torch.float64, "auto"),
    ("res", 0.5, torch.float64, "auto"),
    ("exp", 1.0, torch.float32, "auto"),
    ("res", 0.25, torch.float32, "auto"),
    ("exp", 0.0, torch.float32, "lanczos"),
]


@pytest.mark.parametrize("kind,mu,dtype,method", CASES)
def test_ws_calls_equal_allocating_calls(lib, ba20k, kind, mu, dtype, method):
    n, rp, ci, As = ba20k
    print(f"[gpu] workspace {kind} mu={mu} {dtype} {method}", flush=True)
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci)
    lam = sparse.lambda_max(As)
    param = 1.0 / lam if kind == "exp" else 0.5 / sparse.rho_Z(As, mu)
    b = 16

    def make():
        return lib.Operator(g, mu, kind, param, dtype=dtype, krylov_dim=30, method=method)

    X = torch.tensor(synth.rademacher_block(n, b, 3), dtype=dtype, device="cuda")
    ref_op = make()
    P_ref = ref_op.apply_phi(X)
    L_ref = ref_op.apply_L(X)
    (E_ref,), e_ref = ref_op.expv(X, [1.0], outer_dim=12)

    op = make()  # fresh: walk degrees not cached, so the Laplacian calls compute them in the region
    wP, nP = work_for(op, "apply_phi", b)
    wL, nL = work_for(op, "apply_L", b)
    wE, nE = work_for(op, "expv", b, 12)
    assert nL > nP > 0 and nE > nL
    # outputs from torch before the calls (its caching allocator takes 20 MiB segments)
    P, L, E = torch.empty_like(X), torch.empty_like(X), torch.empty_like(X)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    op.apply_phi_ws(X, wP, out=P)
    op.apply_L_ws(X, wL, out=L)
    (E,), e = op.expv_ws(X, [1.0], wE, outer_dim=12, outs=[E])
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free0 - free1 < (4 << 20), (free0, free1, nE)
    assert torch.equal(P, P_ref) and torch.equal(L, L_ref) and torch.equal(E, E_ref)
    assert e == e_ref
    # after the walk degrees are cached the Laplacian calls need less and still agree
    op.fdeg()
    assert op.workspace_size("apply_L", b) == nP
    L2 = op.apply_L_ws(X, wL)
    assert torch.equal(L2, L_ref)
    # a region reused by another call kind gives the same results
    P2 = op.apply_phi_ws(X, wE)
    assert torch.equal(P2, P_ref)


def test_ws_argument_checks(lib, ba20k):
    n, rp, ci, As = ba20k
    ctx = lib.Context(0)
    g = lib.Graph(ctx, rp, ci)
    op = lib.Operator(g, 0.5, "exp", 1.0 / sparse.lambda_max(As), dtype=torch.float32, krylov_dim=10)
    X = torch.ones((n, 4), dtype=torch.float32, device="cuda")
    Y = torch.empty_like(X)
    need = op.workspace_size("apply_phi", 4)
    small = torch.empty(need - 256, dtype=torch.uint8, device="cuda")
    st = lib.load().wl_apply_phi_ws(op.handle, lib._ptr(X), lib._ptr(Y), 4, lib._ptr(small), need - 256)
    assert st == lib._lib.WL_EINVAL and b"smaller" in lib.load().wl_last_error()
    big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
    st = lib.load().wl_apply_phi_ws(op.handle, lib._ptr(X), lib._ptr(Y), 4, C.c_void_p(big.data_ptr() + 16), need)
    assert st == lib._lib.WL_EINVAL and b"aligned" in lib.load().wl_last_error()
    v = C.c_size_t()
    assert lib.load().wl_workspace_size(op.handle, 7, 4, 0, C.byref(v)) == lib._lib.WL_EINVAL
    arn = lib.Operator(g, 0.5, "exp", 1.0 / sparse.lambda_max(As), dtype=torch.float32, krylov_dim=10,
                       method="arnoldi")
    assert lib.load().wl_workspace_size(arn.handle, 0, 4, 0, C.byref(v)) == lib._lib.WL_EUNSUPPORTED
