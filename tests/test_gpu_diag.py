"""The random-gather probe (wl_gather_probe) that the sparse products' line traffic is
set against: it gathers the rows it is asked for (the sum of its outputs is the sum of
the gathered rows), skips indices outside the table, and rejects bad shapes."""

import ctypes as C

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("row_bytes", [16, 64, 128, 512])
def test_gather_probe_sums_the_gathered_rows(lib, row_bytes):
    print(f"[gpu] gather probe {row_bytes}", flush=True)
    ctx = lib.Context(0)
    rows, count, blocks = 3000, 20011, 64
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    table = torch.randint(-4, 5, (rows, row_bytes // 4), generator=gen, device="cuda").float()
    idx = torch.randint(0, rows, (count,), dtype=torch.int32, device="cuda", generator=gen)
    idx[::97] = rows + 5  # outside the table: skipped
    out = torch.empty(blocks * 256 * 4, dtype=torch.float32, device="cuda")
    ms = C.c_double()
    lib._lib.check(lib.load().wl_gather_probe(ctx.handle, lib._ptr(table), rows, row_bytes, lib._ptr(idx), count,
                                              lib._ptr(out), blocks, 2, C.byref(ms)))
    keep = idx < rows
    ref = table[idx[keep].long()].double().sum()
    assert float(out.double().sum()) == float(ref)  # small integers: exact in FP32
    assert ms.value > 0.0


def test_gather_probe_rejects_bad_shapes(lib):
    ctx = lib.Context(0)
    table = torch.zeros(1024, dtype=torch.float32, device="cuda")
    idx = torch.zeros(16, dtype=torch.int32, device="cuda")
    out = torch.empty(256 * 4, dtype=torch.float32, device="cuda")
    ms = C.c_double()
    for rb in (24, 48, 1024):
        with pytest.raises(lib.WLError, match="EINVAL"):
            lib._lib.check(lib.load().wl_gather_probe(ctx.handle, lib._ptr(table), 16, rb, lib._ptr(idx), 16,
                                                      lib._ptr(out), 1, 1, C.byref(ms)))
