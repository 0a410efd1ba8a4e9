"""Throughput of the SpMM-Krylov evaluation of f(A)V on one MI355X.

Workload (default "ba1m"): Barabasi-Albert graph, n = 1,000,000, m = 5 (seed clique
K_6; 9,999,970 directed nonzeros), unweighted int32 CSR.  All three walk variants:
mu in {0 (all walks), 0.25, 0.5, 0.75 (downweighted, theta = 1 - mu), 1 (NBT)},
each with the exponential (beta = 1/lambda_max, fused recurrence of degree 30) and
the resolvent (alpha = 0.5/rho(Z_mu), 30 block Lanczos steps on the deformed
Laplacian with FP64 tridiagonal evaluation).  V: 16 Rademacher vectors, FP32.

One step = for each of the 10 operators: w = f(A)1 (b = 1) and L V = w*V - f(A)V
(b = 16).  GEdge.vec/s = sum over sparse products of nnz * b, divided by the wall
time of the step (graph upload and spectral scale are outside it), / 1e9.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GEdge·vec/s of SpMM-Krylov f(A)V"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="ba1m", choices=["ba1m"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--krylov", type=int, default=30)
    p.add_argument("--block", type=int, default=16)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device-to-device copy 5 times (reference for HBM counters)")
    return p.parse_args()


def copy_calibration():
    """A plain copy of known size: 5 x (read 1 GiB + write 1 GiB).  Run under the same
    hardware counters as the bench, it gives the factor between counter readings and
    bytes actually moved."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"copy_bytes_each": 2 * src.numel() * 4, "copies": 5, "seconds": dt,
                      "GBps": 5 * 2 * src.numel() * 4 / dt / 1e9}), flush=True)


def measured_traffic(n, m, b):
    """HBM bytes per launch of the dominant kernel from the committed FETCH_SIZE /
    WRITE_SIZE counter runs, scaled by the copy-kernel calibration; None when the
    kernel source changed since the counters were taken or the workload differs."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "k_spmm_recurrence_ba1m_traffic.json")
    src = os.path.join(ROOT, "paper_2601_11338_amd", "csrc", "spmm.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if sha != rec.get("source_sha1") or (n, m, b) != (1000000, 5, 16):
        return None
    return rec["traffic_bytes_per_launch"]


def cpu_baseline(rp, ci, n, lam, X, K):
    """The oracle (sparse FP64 series, eq. qrec) on a bounded sample of the step:
    one of the ten operators (mu = 0.5, exponential), degree K, on 1 + b columns."""
    import numpy as np
    from oracle import sparse

    A = sparse.adjacency(n, rp, ci)
    beta = 1.0 / lam
    coeffs = np.array([beta ** k / math.factorial(k) for k in range(K + 1)])
    t0 = time.perf_counter()
    sparse.series_apply(A, 0.5, coeffs, np.ones((n, 1)))
    sparse.series_apply(A, 0.5, coeffs, X.astype(np.float64))
    dt = time.perf_counter() - t0
    ev = K * A.nnz * (1 + X.shape[1])
    return {
        "value": ev / dt / 1e9,
        "unit": "GEdge·vec/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"1 of 10 operators (mu=0.5, exp, degree {K}) on 1+{X.shape[1]} columns, "
                  f"scipy.sparse single-threaded FP64, {dt:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (multi-GPU is design-only)",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import torch

    import paper_2601_11338_amd as wl
    import synth

    n, m, K, b = 1_000_000, 5, args.krylov, args.block
    log("generating Barabasi-Albert graph")
    rp, ci = synth.barabasi_albert(n, m, seed=2026)
    nnz = int(ci.size)
    X_h = synth.rademacher_block(n, b, seed=3, dtype=np.float32)
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    log(f"graph n={n} nnz={nnz} max_degree={g.info()[2]}")
    g.autotune(torch.float32, b)
    g.autotune(torch.float32, 1)
    lam = g.lambda_max()
    mus = [0.0, 0.25, 0.5, 0.75, 1.0]
    ops = []
    for mu in mus:
        rho = g.spectral_radius(mu)
        log(f"mu={mu}: rho(Z_mu)={rho:.6f} (lambda_max={lam:.6f})")
        ops.append((mu, "exp", wl.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=K)))
        ops.append((mu, "res", wl.Operator(g, mu, "res", 0.5 / rho, dtype=torch.float32, krylov_dim=K,
                                           rho_hint=rho)))
    X = torch.tensor(X_h, device="cuda")
    ones = torch.ones((n, 1), dtype=torch.float32, device="cuda")
    W = torch.empty((n, 1), dtype=torch.float32, device="cuda")
    Y = torch.empty((n, b), dtype=torch.float32, device="cuda")
    for _, _, op in ops:
        op.fdeg()  # cached w for the Laplacian finish

    def step():
        for _, _, op in ops:
            op.apply_phi(ones, out=W)
            op.apply_L(X, out=Y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    rec = ctx.kernel_stats(0)
    lan = ctx.kernel_stats(1)
    ctx.set_profiling(False)
    edge_vec = len(ops) * K * nnz * (1 + b)
    value = edge_vec / (ms * 1e-3) / 1e9
    # dominant kernel: fused recurrence step on the 16-wide block
    launches, kms, kbytes = rec
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    lan_avg = lan[1] / max(lan[0], 1)
    log(f"recurrence kernel: {launches} launches, avg {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic; "
        f"Lanczos operator kernel: {lan[0]} launches, avg {lan_avg * 1e3:.1f} us")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "GEdge·vec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"barabasi-albert n={n} m={m} nnz={nnz}; mu in {mus} x {{exp beta=1/lambda_max, "
                        f"res alpha=0.5/rho(Z_mu)}}; b={b} Rademacher + f(A)1; Krylov dim {K}; FP32 vectors, "
                        f"FP64 coefficients",
            "n": n,
            "nnz": nnz,
            "block": b,
            "krylov_dim": K,
            "operators": len(ops),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(n, m, b),
            "kernel": "k_spmm<float,4,4,G> fused recurrence step (b=16)",
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(rp, ci, n, lam, X_h, K)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
