"""The block Krylov primitives (tall-skinny Gram and block update) against numpy,
through the C ABI.  Inputs are FP32-representable so both sides see identical
values; Grams accumulate in FP64 on both sides."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx(lib):
    return lib.Context(0)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bx,by", [(1, 1), (3, 3), (4, 4), (8, 8), (16, 16), (20, 20), (32, 32), (64, 64), (16, 5)])
@pytest.mark.parametrize("n,nblk", [(1, 1), (7, 1), (1000, 3), (50001, 1)])
def test_block_gram(ctx, lib, dtype, bx, by, n, nblk):
    print(f"[gpu] gram {dtype} {bx}x{by} n={n} nblk={nblk}", flush=True)
    rng = np.random.default_rng(bx * 100 + by + n)
    X = f32(rng.standard_normal((nblk * n, bx)))
    Y = f32(rng.standard_normal((n, by)))
    td = torch.float32 if dtype == "f32" else torch.float64
    G = lib.block_gram(ctx, torch.tensor(X, dtype=td, device="cuda"), torch.tensor(Y, dtype=td, device="cuda"), nblk)
    ref = np.vstack([X[k * n:(k + 1) * n].T @ Y for k in range(nblk)])
    np.testing.assert_allclose(G, ref, rtol=1e-11, atol=1e-11 * np.sqrt(n))


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("b", [1, 3, 4, 8, 16, 32, 64])
@pytest.mark.parametrize("nblk", [1, 3, 13, 25])
@pytest.mark.parametrize("with_y", [False, True])
def test_block_update(ctx, lib, dtype, b, nblk, with_y):
    n = 4099
    print(f"[gpu] update {dtype} b={b} nblk={nblk} y={with_y}", flush=True)
    rng = np.random.default_rng(b + 10 * nblk)
    X = f32(rng.standard_normal((nblk * n, b)))
    Cm = rng.standard_normal((nblk * b, b))
    Yin = f32(rng.standard_normal((n, b)))
    td = torch.float32 if dtype == "f32" else torch.float64
    Xd = torch.tensor(X, dtype=td, device="cuda")
    Yd = torch.tensor(Yin, dtype=td, device="cuda") if with_y else None
    out, G = lib.block_update(ctx, Xd, Cm, Yin=Yd, alpha=0.5, beta=-1.25, nblk=nblk, want_gram=True)
    ref = -1.25 * sum(X[k * n:(k + 1) * n] @ Cm[k * b:(k + 1) * b] for k in range(nblk))
    if with_y:
        ref = ref + 0.5 * Yin
    got = out.cpu().numpy().astype(np.float64)
    tol = 2e-5 if dtype == "f32" else 1e-12
    np.testing.assert_allclose(got, ref, rtol=tol, atol=tol * np.abs(ref).max())
    np.testing.assert_allclose(G, got.T @ got, rtol=1e-9, atol=1e-9 * np.abs(got.T @ got).max())


@pytest.mark.parametrize("b", [4, 16, 32])
def test_block_update_in_place(ctx, lib, b):
    n = 3000
    rng = np.random.default_rng(b)
    X = f32(rng.standard_normal((n, b)))
    Cm = rng.standard_normal((b, b))
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    lib.block_update(ctx, Xd, Cm, out=Xd)
    np.testing.assert_allclose(Xd.cpu().numpy(), X @ Cm, rtol=2e-5, atol=2e-5 * np.abs(X @ Cm).max())


@pytest.mark.parametrize("nblk", [5, 13, 30])
def test_block_update_out_is_an_input_block(ctx, lib, nblk):
    """Out aliasing the first of many input blocks (32-wide FP32: combinations longer
    than one launch holds run on the general kernel then) and the last one."""
    n, b = 2500, 32
    rng = np.random.default_rng(nblk)
    X = f32(rng.standard_normal((nblk * n, b)))
    Cm = rng.standard_normal((nblk * b, b))
    ref = sum(X[k * n:(k + 1) * n] @ Cm[k * b:(k + 1) * b] for k in range(nblk))
    for k_out in (0, nblk - 1):
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        out = Xd[k_out * n:(k_out + 1) * n]
        lib.block_update(ctx, Xd, Cm, nblk=nblk, out=out)
        np.testing.assert_allclose(out.cpu().numpy(), ref, rtol=2e-5, atol=2e-5 * np.abs(ref).max())
