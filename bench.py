"""Throughput of the SpMM-Krylov evaluation of f(A)V on one MI355X.

Workload (default "ba1m"): Barabasi-Albert graph, n = 1,000,000, m = 5 (seed clique
K_6; 9,999,970 directed nonzeros), unweighted int32 CSR.  All three walk variants:
mu in {0 (all walks), 0.25, 0.5, 0.75 (downweighted, theta = 1 - mu), 1 (NBT)},
each with the exponential (beta = 1/lambda_max, fused recurrence of degree 30) and
the resolvent (alpha = 0.5/rho(Z_mu), 30 block Lanczos steps on the deformed
Laplacian with FP64 tridiagonal evaluation).  V: 16 Rademacher vectors, FP32.

One step = for each of the 10 operators: w = f(A)1 (b = 1) and L V = w*V - f(A)V
(b = 16).  GEdge.vec/s = sum over sparse products of nnz * b, divided by the wall
time of the step (graph upload and spectral scale are outside it), / 1e9.  The five
exponential operators run side by side (walk degrees in one pass, L V of four in one
64-wide pass); the five resolvent operators (block Lanczos) run on further streams
concurrently with them (--streams, one library context per stream).
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
    p.add_argument("--workload", default="ba1m", choices=["ba1m", "batch512", "cv-rmat22", "expv-rmat25", "markov-ba1m", "arp-road2m", "arnoldi-ba1m",
                            "amg-road2m"],
                   help="ba1m: one Barabasi-Albert graph, n=10^6 (default); batch512: 512 SBM / "
                        "configuration-model graphs, diffusion and return probabilities in one batch; "
                        "cv-rmat22: learned control variate trained on 200 small graphs, diagonal "
                        "error versus probes on an R-MAT scale-22 graph; expv-rmat25: diffusion of 32 "
                        "sparse initial conditions on an R-MAT scale-25 graph (33.5M nodes)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--separate", action="store_true",
                   help="ba1m: evaluate every operator on its own (no side-by-side series operators)")
    p.add_argument("--no-pack", action="store_true",
                   help="ba1m: walk degrees in passes of their own (four series operators side by side, the "
                        "resolvent operators as Lanczos pairs) instead of riding beside the blocks")
    p.add_argument("--res-layout", choices=["pairs", "packed"], default="pairs",
                   help="ba1m: resolvent operators as two Lanczos pairs (32 wide), one single operator and their "
                        "walk degrees as single-column processes on three streams (pairs), or all five with "
                        "their walk degrees in one 96-wide block (packed)")
    p.add_argument("--shapes", default="",
                   help="ba1m, markov-ba1m: fixed sparse-product launch shapes width:lanes:threshold,... instead of autotuning "
                        "(e.g. to take hardware counters on the shapes a timed run chose)")
    p.add_argument("--streams", type=int, default=4,
                   help="ba1m: independent operator groups run concurrently on this many streams (one library "
                        "context per stream, all borrowing one device CSR)")
    p.add_argument("--krylov", type=int, default=30)
    p.add_argument("--arnoldi-steps", type=int, default=20, help="Krylov dimension of the arnoldi-ba1m workload")
    p.add_argument("--block", type=int, default=16)
    p.add_argument("--gather-ceiling", action="store_true",
                   help="only measure the machine ceilings: random whole-row gathers from a 10^6-row table "
                        "(wl_gather_probe) at several row sizes, a plain device copy and a plain read")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device-to-device copy 5 times (reference for HBM counters)")
    p.add_argument("--summarize", metavar="DIR",
                   help="only summarise a rocprofv3 output folder (kernel trace or counter CSVs): per kernel, the "
                        "number of dispatches, the mean over all and over the last --last dispatches")
    p.add_argument("--last", type=int, default=358, help="dispatches per kernel averaged by --summarize")
    p.add_argument("--window-ms", type=float, default=0.0,
                   help="--summarize of a kernel trace: only the dispatches of the trace's last WINDOW_MS "
                        "milliseconds (the last step when nothing runs after it), with the time the GPU was "
                        "busy and the longest idle gaps")
    p.add_argument("--no-reference", action="store_true",
                   help="arp-road2m: skip the standard-Laplacian estimate after the timed region")
    return p.parse_args()


def summarize(folder, last):
    """Per-kernel figures from rocprofv3 CSV output: durations in us for a kernel trace,
    the counter value for a counter collection.  The last dispatches of a kernel are the
    last step(s) of the command, after autotuning and warm-up."""
    import collections
    import csv
    import glob

    for f in sorted(glob.glob(os.path.join(folder, "**", "*.csv"), recursive=True)):
        trace = f.endswith("kernel_trace.csv")
        if not (trace or f.endswith("counter_collection.csv")):
            continue
        per = collections.defaultdict(list)
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if trace:
                    per[r["Kernel_Name"]].append((int(r["Start_Timestamp"]), (int(r["End_Timestamp"]) -
                                                                              int(r["Start_Timestamp"])) / 1e3))
                else:
                    key = f"{r['Counter_Name']} {r['Kernel_Name']}"
                    per[key].append((int(r.get("Dispatch_Id") or 0), float(r["Counter_Value"])))
        print(f"# {os.path.relpath(f, folder)}: " + ("duration us" if trace else "counter value per dispatch"))
        rows = []
        for k, v in per.items():
            v.sort()
            vals = [x for _, x in v]
            tail = vals[-last:]
            rows.append((sum(vals) if trace else len(vals), k, len(vals), sum(vals) / len(vals), len(tail),
                         sum(tail) / len(tail)))
        rows.sort(reverse=True)
        for _, k, nv, avg, nt, avgt in rows[:30]:
            print(f"{nv:7d} x {avg:12.1f} | last {nt:5d}: {avgt:12.1f}  {k[:120]}")


def summarize_window(folder, window_ms):
    """The dispatches of a kernel trace that start within its last window_ms: per kernel
    the total and mean duration, the union of the dispatch intervals (GPU busy) and the
    longest gaps between them with the kernels on either side."""
    import collections
    import csv
    import glob

    for f in sorted(glob.glob(os.path.join(folder, "**", "*kernel_trace.csv"), recursive=True)):
        rows = []
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r["Kernel_Name"]))
        if not rows:
            continue
        rows.sort()
        t0 = max(e for _, e, _ in rows) - window_ms * 1e6
        rows = [x for x in rows if x[0] >= t0]
        per = collections.defaultdict(lambda: [0, 0.0])
        busy, last_end, gaps, prev = 0.0, None, [], None
        for st, en, k in rows:
            per[k][0] += 1
            per[k][1] += (en - st) / 1e6
            if last_end is None:
                busy += (en - st) / 1e6
            else:
                if st > last_end:
                    gaps.append(((st - last_end) / 1e6, prev, k))
                busy += max(0, en - max(st, last_end)) / 1e6
            last_end = en if last_end is None else max(last_end, en)
            prev = k
        print(f"# {os.path.relpath(f, folder)}: last {window_ms:.1f} ms, {len(rows)} dispatches, GPU busy "
              f"{busy:.1f} ms, idle {window_ms - busy:.1f} ms")
        for k, (c, ms) in sorted(per.items(), key=lambda x: -x[1][1])[:30]:
            print(f"{ms:9.3f} ms {c:7d} x {ms / c * 1e3:10.1f} us  {k[:110]}")
        gaps.sort(reverse=True)
        print(f"# longest idle gaps (of {len(gaps)}, {sum(g for g, _, _ in gaps):.1f} ms in all)")
        for g, a, b in gaps[:12]:
            print(f"{g:8.3f} ms after {a[:60]}  before {b[:60]}")


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


def gather_ceiling():
    """The machine ceilings the sparse products are set against: random gathers of whole
    rows (16 to 512 bytes) of a 10^6-row table, 10^7 gathers per launch with uniformly
    drawn rows (wl_gather_probe), the same probe reading the table in order, and a plain
    copy and sum of 2 GiB (torch kernels)."""
    import ctypes as C

    import torch

    import paper_2601_11338_amd as wl

    ctx = wl.Context(0)
    rows, count = 1_000_000, 10_000_000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    idx = torch.randint(0, rows, (count,), dtype=torch.int32, device="cuda", generator=gen)
    table = torch.rand(rows * 128, dtype=torch.float32, device="cuda", generator=gen)  # rows of up to 512 B
    blocks_max = 32768
    out = torch.empty(blocks_max * 256 * 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    res = {"rows": rows, "gathers_per_launch": count, "gather": []}
    for rb in (16, 64, 128, 256, 512):
        for blocks in (8192, blocks_max):
            ms = C.c_double()
            wl._lib.check(wl.load().wl_gather_probe(ctx.handle, wl._ptr(table), rows, rb, wl._ptr(idx), count,
                                                    wl._ptr(out), blocks, 10, C.byref(ms)))
            t = ms.value * 1e-3
            lines = -(-rb // 128)
            res["gather"].append({"row_bytes": rb, "blocks": blocks, "us": t * 1e6,
                                  "useful_GBps": count * rb / t / 1e9,
                                  "line_GBps": count * lines * 128 / t / 1e9})
            log(f"gather {rb:4d} B rows, {blocks} blocks: {t * 1e6:8.1f} us, useful {count * rb / t / 1e9:6.0f} GB/s, "
                f"128-byte lines {count * lines * 128 / t / 1e9:6.0f} GB/s")
    # the same probe with rows in order: a plain coalesced read of the table
    seq = torch.arange(rows, dtype=torch.int32, device="cuda")
    ms = C.c_double()
    wl._lib.check(wl.load().wl_gather_probe(ctx.handle, wl._ptr(table), rows, 512, wl._ptr(seq), rows, wl._ptr(out),
                                            8192, 10, C.byref(ms)))
    res["read_in_order_GBps"] = rows * 512 / (ms.value * 1e-3) / 1e9
    log(f"the table's rows in order (512 MB read): {res['read_in_order_GBps']:.0f} GB/s")
    del table, out, seq
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    a.record()
    for _ in range(5):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    res["copy_GBps"] = 5 * 2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9
    s_ = src.sum()
    a.record()
    for _ in range(5):
        s_ = src.sum()
    b.record()
    torch.cuda.synchronize()
    res["sum_GBps"] = 5 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9
    log(f"copy (read + write of 2 GiB) {res['copy_GBps']:.0f} GB/s, sum of 2 GiB {res['sum_GBps']:.0f} GB/s")
    print(json.dumps(res), flush=True)


def machine_ceilings(ctx, row_bytes):
    """This box's ceilings beside the 8 TB/s specification, measured in the run (outside
    the timed region, well under a second): a device-to-device copy of 2 GiB (read +
    write) and random whole-line gathers of row_bytes-byte rows (10^7 uniformly drawn rows
    of a 10^6-row table, wl_gather_probe), as 128-byte lines per second."""
    import ctypes as C

    import torch

    import paper_2601_11338_amd as wl

    rows, count = 1_000_000, 10_000_000
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    idx = torch.randint(0, rows, (count,), dtype=torch.int32, device="cuda", generator=gen)
    table = torch.rand(rows * row_bytes // 4, dtype=torch.float32, device="cuda", generator=gen)
    out = torch.empty(8192 * 256 * 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    ms = C.c_double()
    wl._lib.check(wl.load().wl_gather_probe(ctx.handle, wl._ptr(table), rows, row_bytes, wl._ptr(idx), count,
                                            wl._ptr(out), 8192, 5, C.byref(ms)))
    lines = -(-row_bytes // 128)
    gather = count * lines * 128 / (ms.value * 1e-3) / 1e9
    del table, out, idx
    src = torch.ones(1 << 29, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    dst.copy_(src)
    a.record()
    for _ in range(3):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    copy = 3 * 2 * src.numel() * 4 / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return {"copy_GBps": copy, "gather_row_bytes": row_bytes, "gather_line_GBps": gather}


def measured_traffic(n, m, width, lanes):
    """HBM bytes per launch of the dominant kernel (the sparse product at this block
    width) from the committed FETCH_SIZE / WRITE_SIZE counter runs, scaled by the
    copy-kernel calibration; None when no such record exists, the kernel source changed
    since the counters were taken, the workload differs or the autotuner picked another
    launch shape."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_spmm_w{width}_ba1m_traffic.json")
    src = os.path.join(ROOT, "paper_2601_11338_amd", "csrc", "spmm.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if sha != rec.get("source_sha1") or (n, m) != (1000000, 5) or rec.get("lanes_per_row") != lanes:
        return None
    return rec["traffic_bytes_per_launch"]


def traffic_record(name, lanes=None):
    """HBM bytes per launch of a workload's dominant kernel from its committed counter
    record (profiles/<name>_traffic.json: FETCH_SIZE / WRITE_SIZE of one run of the
    workload, scaled by the copy-kernel calibration); None when there is no record, the
    kernel source changed since the counters were taken, or (lanes given) the autotuner
    picked another launch shape."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{name}_traffic.json")
    src = os.path.join(ROOT, "paper_2601_11338_amd", "csrc", "spmm.hip")
    try:
        rec = json.load(open(path))
        sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    except (OSError, ValueError):
        return None
    if sha != rec.get("source_sha1"):
        return None
    if lanes is not None and rec.get("lanes_per_row") is not None and rec["lanes_per_row"] != lanes:
        return None
    return rec["traffic_bytes_per_launch"]


def with_nproc(out):
    """The host's CPU count beside the CPU baseline's thread count (cores)."""
    cb = out.get("cpu_baseline")
    if isinstance(cb, dict):
        cb.setdefault("nproc", os.cpu_count())
    return out


def cpu_baseline(rp, ci, n, lam, X, K):
    """The oracle (sparse FP64 series, eq. qrec) on a bounded sample of the step:
    one of the ten operators (mu = 0.5, exponential), degree K, on 1 + b columns."""
    import numpy as np
    from oracle import krylov, sparse

    A = sparse.adjacency(n, rp, ci)
    beta = 1.0 / lam
    coeffs = krylov.exp_coefficients(beta, K)
    nt = krylov.threads()
    t0 = time.perf_counter()
    reps = 0
    while True:  # whole operator evaluations until about 10 s of host time
        krylov.series_apply(A, 0.5, coeffs, np.ones((n, 1)))
        krylov.series_apply(A, 0.5, coeffs, X.astype(np.float64))
        reps += 1
        if time.perf_counter() - t0 > 10.0 or reps == 8:
            break
    dt = time.perf_counter() - t0
    ev = reps * K * A.nnz * (1 + X.shape[1])
    return {
        "value": ev / dt / 1e9,
        "unit": "GEdge·vec/s",
        "cores": nt,
        "nproc": os.cpu_count(),
        "kind": "oracle",
        "sample": f"{reps} evaluation(s) of 1 of the 10 operators (mu=0.5, exp, degree {K}) on 1+{X.shape[1]} "
                  f"columns, FP64 series with scipy.sparse products split over {nt} host threads, {dt:.1f} s",
    }


def _gen_spec(spec):
    import synth
    return synth.graph_from_spec(spec)


def run_batch512(args):
    """512 graphs (SBM with 4..32 blocks and p_in/p_out = 20, power-law configuration
    model with exponent 2.5; sizes log-uniform on [1e3, 2e5]) with mixed variants:
    graph i has mu = (0, .25, .5, .75, 1)[i % 5], the exponential (beta = 1/lambda_max)
    or the resolvent (alpha = 0.5/lambda_max, which is below 1/rho(Z_mu) for every mu)
    alternating every five graphs, and t = (0.1, 1, 10)[i % 3].  One step = one batched
    diffusion exp(-t_g L_g) U0_g with 8 Gaussian probes per graph and 30 outer block
    Lanczos steps, plus every graph's Nystrom return probability p_hat(t_g)."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2601_11338_amd as wl
    import synth

    count, b, K_out = 512, 8, args.krylov
    specs = synth.batch_specs(count, seed=2026)
    log(f"generating {count} graphs")
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        csrs = list(ex.map(_gen_spec, specs, chunksize=8))
    ctx = wl.Context(0)
    graphs = [wl.Graph(ctx, rp, ci) for rp, ci in csrs]
    nnz = np.array([g.nnz for g in graphs], dtype=np.int64)
    log(f"graphs uploaded: sum n={sum(g.n for g in graphs)} sum nnz={int(nnz.sum())}")
    mus = [0.0, 0.25, 0.5, 0.75, 1.0]
    descs, ts = [], []
    for i, g in enumerate(graphs):
        lam = g.lambda_max()
        mu = mus[i % 5]
        if (i // 5) % 2 == 0:
            descs.append({"mu": mu, "func": "exp", "param": 1.0 / lam})
        else:
            descs.append({"mu": mu, "func": "res", "param": 0.5 / lam, "rho_hint": lam})
        ts.append((0.1, 1.0, 10.0)[i % 3])
    log("spectral scales done; building the batch")
    batch = wl.Batch(ctx, graphs, descs, tol=1e-8)
    batch.autotune(b)
    Kg = batch.series_degrees.astype(np.int64)
    offs = np.append(batch.offsets, batch.total_rows)
    npad = np.diff(offs)
    log(f"batch rows {batch.total_rows}, series degrees {Kg.min()}..{Kg.max()} (mean {Kg.mean():.1f}); "
        f"XCD-grouped tile order chosen: {batch.xcd_grouped}")
    # 8 Gaussian probes per graph (Philox), zero on the padding rows
    U0 = wl.probes(ctx, batch.total_rows, b, seed=11)
    keep = torch.zeros(batch.total_rows, dtype=torch.bool, device="cuda")
    for o, g in zip(batch.offsets, graphs):
        keep[int(o):int(o) + g.n] = True
    U0 = (U0 * keep[:, None]).contiguous()
    Y = torch.empty_like(U0)

    def step():
        return batch.expv(U0, ts, outer_dim=K_out, out=Y)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, p_hat, p_err = step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    rec = ctx.kernel_stats(0)
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    edge_vec = K_out * float((Kg * nnz).sum()) * b
    value = edge_vec / (ms * 1e-3) / 1e9
    # algorithmic bytes of the recurrence launches of one inner product, counting only
    # the rows of graphs still inside their series (the others are skipped)
    alg = 0.0
    for k in range(1, int(Kg.max()) + 1):
        act = Kg >= k
        streams = 4 if k == 1 else 5
        alg += float((4 * nnz[act] + 4 * npad[act] + 4 * b * npad[act] * streams).sum())
        fin = Kg == k
        alg += float((4 * b * npad[fin] + 4 * npad[fin]).sum())
    alg *= K_out * args.steps
    launches, kms, _ = rec
    achieved = alg / (kms * 1e-3) / 1e9 if kms > 0 else 0.0
    log(f"recurrence kernel: {launches} launches, avg {kms / max(launches, 1) * 1e3:.1f} us, "
        f"{achieved:.0f} GB/s algorithmic; mean p_hat {np.mean(p_hat):.4f}")
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
            "workload": f"batch of {count} graphs (SBM 4..32 blocks p_in/p_out=20, power-law CM exponent 2.5; "
                        f"n log-uniform 1e3..2e5); mixed mu/f, t in {{0.1,1,10}}; b={b} Gaussian probes; "
                        f"outer Krylov dim {K_out}; inner series to 1e-8; p_hat per graph",
            "graphs": count,
            "sum_n": int(sum(g.n for g in graphs)),
            "sum_nnz": int(nnz.sum()),
            "block": b,
            "krylov_dim": K_out,
            "series_degree_max": int(Kg.max()),
            "xcd_grouped_tiles": batch.xcd_grouped,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record("k_spmm_b8_batch512"),
            "kernel": "k_spmm batched recurrence step (b=8, per-graph coefficient table)",
            "avg_launch_us": kms / max(launches, 1) * 1e3,
            "alg_bytes_per_launch": alg / max(launches, 1),
        },
        "p_hat_mean": float(np.mean(p_hat)),
        "p_err_mean": float(np.mean(p_err)),
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline_batch(csrs, descs, b)
    return out


def cpu_baseline_batch(csrs, descs, b, budget_s=15.0):
    """The oracle's sparse FP64 series (eq. qrec) applied to a b-column block, graph
    after graph, until the time budget is spent: the inner product of one outer step."""
    import numpy as np
    from oracle import sparse

    done_ev, t_used, graphs = 0.0, 0.0, 0
    for (rp, ci), d in zip(csrs, descs):
        n = len(rp) - 1
        A = sparse.adjacency(n, rp, ci)
        K = 30
        if d["func"] == "exp":
            coeffs = np.array([d["param"] ** k / math.factorial(k) for k in range(K + 1)])
        else:
            coeffs = np.array([d["param"] ** k for k in range(K + 1)])
        X = np.ones((n, b))
        t0 = time.perf_counter()
        sparse.series_apply(A, d["mu"], coeffs, X)
        t_used += time.perf_counter() - t0
        done_ev += K * A.nnz * b
        graphs += 1
        if t_used > budget_s:
            break
    return {
        "value": done_ev / t_used / 1e9,
        "unit": "GEdge·vec/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"degree-30 series on 8 columns for the first {graphs} graphs of the batch, "
                  f"scipy.sparse single-threaded FP64, {t_used:.1f} s",
    }


def run_expv_rmat25(args):
    """Diffusion on R-MAT scale 25 (edge factor 16, a = 0.57, b = c = 0.19; 33.5M
    nodes, about 1e9 symmetric nonzeros): exp(-t L) U0 for t in {0.1, 1, 10} with
    L the walk Laplacian of mu = 0.5 (theta = 0.5) and the exponential (beta =
    1/lambda_max, inner series degree from the tail bound at 1e-9), U0 = 32 sparse
    probability vectors (16 random non-isolated nodes each), 40 outer block Lanczos
    steps, FP32 vectors with FP64 coefficients.  One step = one wl_expv call for the
    three times (one Krylov basis serves all t)."""
    import torch

    import paper_2601_11338_amd as wl
    import synth

    b, K_out, ts = 32, args.krylov if args.krylov != 30 else 40, [0.1, 1.0, 10.0]
    log("generating R-MAT scale 25 on the device")
    rp, ci = synth.rmat_device(25, 16, 0.57, 0.19, 0.19, seed=2025)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()  # the Krylov basis (about 176 GB) is allocated by the library
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    n, nnz = g.n, g.nnz
    log(f"graph n={n} nnz={nnz} max_degree={g.info()[2]}")
    g.autotune(torch.float32, b)
    lam = g.lambda_max()
    op = wl.Operator(g, 0.5, "exp", 1.0 / lam, dtype=torch.float32, tol=1e-9)
    K_in, _ = op.info()
    log(f"lambda_max={lam:.4f}; inner series degree {K_in}")
    deg = rp[1:] - rp[:-1]
    pool = torch.nonzero(deg > 0).flatten()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(25)
    U0 = torch.zeros((n, b), dtype=torch.float32, device="cuda")
    for j in range(b):
        sel = pool[torch.randperm(pool.numel(), generator=gen, device="cuda")[:16]]
        U0[sel, j] = 1.0 / 16
    del pool, deg
    outs = [torch.empty_like(U0) for _ in ts]
    op.fdeg()

    def step():
        return op.expv(U0, ts, outer_dim=K_out, outs=outs)

    for _ in range(args.warmup):
        step()
        log("warm-up step done")
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, err = step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done; a-posteriori errors {['%.2e' % e for e in err]}")
    t1 = time.perf_counter()
    rec = ctx.kernel_stats(0)
    oth = ctx.kernel_stats(2)
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    # inner products: K_in sparse products on b columns per outer step
    edge_vec = K_out * K_in * float(nnz) * b
    value = edge_vec / (ms * 1e-3) / 1e9
    launches, kms, kbytes = rec
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    mass = [float(o.sum()) / float(U0.sum()) for o in outs]
    log(f"recurrence kernel: {launches} launches, avg {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic; "
        f"first-step kernel: {oth[0]} launches; mass ratio {mass}")
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        u0 = U0[:, 0].double().cpu().numpy()[:, None]
        del outs
        cpu = cpu_baseline_expv(rp.cpu().numpy(), ci.cpu().numpy(), n, 0.5, 1.0 / lam, K_in, K_out, b, u0)
    return {
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
            "workload": f"R-MAT scale 25 ef 16 (a=.57 b=c=.19) n={n} nnz={nnz}; mu=0.5 exp beta=1/lambda_max "
                        f"(inner degree {K_in}); exp(-tL)U0 for t in {ts}, U0 32 sparse probability vectors; "
                        f"outer Krylov dim {K_out}; FP32 vectors, FP64 coefficients",
            "n": n,
            "nnz": nnz,
            "block": b,
            "krylov_dim": K_out,
            "inner_degree": K_in,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record("k_spmm_w32_expv_rmat25", g.shape(torch.float32, 32)[0]),
            "kernel": "k_spmm fused recurrence step (b=32)",
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
        },
        "mass_ratio": mass,
        "cpu_baseline": cpu,
    }


def cpu_baseline_expv(rp, ci, n, mu, beta, K_in, K_out, b, u0, degree=4):
    """The oracle's sparse FP64 series (eq. qrec, row-chunked threaded products) on one
    of the 32 columns, cut to its first few products: the GPU step applies the degree
    K_in series K_out times to 32 columns; the rate per edge-vector is taken as what one
    full step would see on the host (the products dominate; the outer Lanczos' vector
    work is not timed)."""
    from oracle import krylov, sparse

    A = sparse.adjacency(n, rp, ci)
    nt = krylov.threads()
    coeffs = krylov.exp_coefficients(beta, degree)
    t0 = time.perf_counter()
    krylov.series_apply(A, mu, coeffs, u0)
    dt = time.perf_counter() - t0
    ev = degree * float(A.nnz)
    full = K_out * K_in * float(A.nnz) * b / (ev / dt)
    return {"value": ev / dt / 1e9, "unit": "GEdge·vec/s", "cores": nt, "nproc": os.cpu_count(), "kind": "oracle",
            "sample": f"FP64 series of degree {degree} (of the GPU's {K_in}) on 1 of the {b} columns, scipy.sparse "
                      f"products split over {nt} host threads, {dt:.1f} s; at this rate one step ({K_out} outer "
                      f"products x {K_in} inner x {b} columns) would take {full / 3600:.1f} h"}


MLP_SHAPES = [(64, 8), (64,), (64, 64), (64,), (1, 64), (1,)]


def run_markov_ba1m(args):
    """Discrete-time diffusion on the BA graph of the default workload (n = 1e6, m = 5):
    the chain P = diag(w)^{-1} phi of the nonbacktracking exponential (mu = 1, beta =
    1/lambda_max, series degree from the tail bound at 1e-9), the operator whose chain
    explores a tree most widely in the paper's tree experiment.  One step = 20 steps of
    the chain from 16 starting nodes (point masses, FP32) + its stationary distribution
    + its spectral gap (Lanczos, 60 steps, on the symmetrised chain)."""
    import numpy as np
    import torch

    import paper_2601_11338_amd as wl
    import synth

    n, m, b, chain, gap_dim = 1_000_000, 5, 16, 20, 60
    log("generating Barabasi-Albert graph")
    rp, ci = synth.barabasi_albert(n, m, seed=2026)
    nnz = int(ci.size)
    starts = np.random.default_rng(590).choice(n, size=b, replace=False)
    P0_h = synth.spike_block(n, starts, dtype=np.float32)
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    if args.shapes:
        for item in args.shapes.split(","):
            w_, l_, t_ = (int(x) for x in item.split(":"))
            g.set_shape(torch.float32, w_, l_, t_)
    else:
        for w_ in (b, 1):
            g.autotune(torch.float32, w_)
    log("launch shapes width:lanes:threshold " +
        ",".join(f"{w_}:{g.shape(torch.float32, w_)[0]}:{g.shape(torch.float32, w_)[1]}" for w_ in (b, 1)))
    lam = g.lambda_max()
    op = wl.Operator(g, 1.0, "exp", 1.0 / lam, dtype=torch.float32, tol=1e-9)
    K_in, _ = op.info()
    log(f"graph n={n} nnz={nnz}; lambda_max={lam:.4f}; series degree {K_in}")
    P0 = torch.tensor(P0_h, device="cuda")
    Pk = torch.empty_like(P0)
    pi = torch.empty(n, dtype=torch.float32, device="cuda")
    op.fdeg()  # w, cached by the operator

    def step():
        op.markov_step(P0, steps=chain, out=Pk)
        op.markov_stationary(out=pi)
        return op.markov_gap(outer_dim=gap_dim, seed=7)

    for _ in range(args.warmup):
        step()
        log("warm-up step done")
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        l2, lmin, gap = step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done; lambda_2={l2:.6f} lambda_min={lmin:.6f} gap={gap:.6f}")
    t1 = time.perf_counter()
    rec = ctx.kernel_stats(0)   # series steps on the 16 distributions
    oth = ctx.kernel_stats(2)   # first steps and the single-vector products of the gap
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    # every application of phi is K_in sparse products: chain * b columns for the
    # steps and gap_dim single columns for the gap
    edge_vec = K_in * float(nnz) * (chain * b + gap_dim)
    value = edge_vec / (ms * 1e-3) / 1e9
    launches, kms, kbytes = rec
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    mass = [float(x) for x in Pk.sum(dim=0).cpu()]
    tv = float((Pk - pi[:, None]).abs().sum(dim=0).max()) / 2
    log(f"series kernel: {launches} launches, avg {avg_ms * 1e3:.1f} us, {achieved:.0f} GB/s algorithmic; "
        f"other: {oth[0]} launches, {oth[1]:.1f} ms; mass {min(mass):.6f}..{max(mass):.6f}; "
        f"max TV distance to pi after {chain} steps {tv:.4f}")
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
            "workload": f"discrete-time diffusion on barabasi-albert n={n} m={m} nnz={nnz}: chain of the "
                        f"mu=1 exp (beta=1/lambda_max, series degree {K_in}); {chain} chain steps from {b} "
                        f"starting nodes + stationary distribution + spectral gap (Lanczos dim {gap_dim}); "
                        f"FP32 vectors, FP64 coefficients",
            "n": n,
            "nnz": nnz,
            "block": b,
            "chain_steps": chain,
            "gap_krylov_dim": gap_dim,
            "inner_degree": K_in,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record("k_spmm_w16_markov_ba1m", g.shape(torch.float32, b)[0]),
            "kernel": f"k_spmm fused recurrence step (b={b})",
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
            "other_kernels": [{"what": "first steps and single-vector products of the gap", "launches": oth[0],
                               "total_ms": oth[1],
                               "achieved": oth[2] / (oth[1] * 1e-3) / 1e9 if oth[1] else 0.0}],
        },
        "gap": {"lambda_2": l2, "lambda_min": lmin, "gap": gap},
        "mass": [min(mass), max(mass)],
        "tv_to_stationary": tv,
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline_markov(rp, ci, n, lam, K_in, P0_h)
    return out


def cpu_baseline_markov(rp, ci, n, lam, K, P0):
    """The oracle (sparse FP64 series, eq. qrec) on a bounded sample of the step: the
    walk degrees w and two chain steps p <- phi (p ./ w) on the 16 distributions."""
    import numpy as np
    from oracle import sparse

    A = sparse.adjacency(n, rp, ci)
    beta = 1.0 / lam
    coeffs = np.array([beta ** k / math.factorial(k) for k in range(K + 1)])
    t0 = time.perf_counter()
    w = sparse.series_apply(A, 1.0, coeffs, np.ones((n, 1)))
    X = P0.astype(np.float64)
    for _ in range(2):
        X = sparse.series_apply(A, 1.0, coeffs, X / w)
    dt = time.perf_counter() - t0
    ev = K * A.nnz * (1 + 2 * P0.shape[1])
    return {
        "value": ev / dt / 1e9,
        "unit": "GEdge·vec/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"walk degrees + 2 chain steps on {P0.shape[1]} distributions (mu=1, exp, degree {K}), "
                  f"scipy.sparse single-threaded FP64, {dt:.1f} s",
    }


def run_arp_road2m(args):
    """Average return probability by Alg. 1 on a road-network stand-in (a 1400 x 1400
    lattice with each edge kept with probability 0.7: n = 1.96e6, mean degree 2.8, the
    size and degree of roadNet-CA) for the nonbacktracking resolvent Laplacian
    (mu = 1, alpha = 1/(1 + rho(Z)), the paper's large-graph setting): M = 30 Gaussian
    probes, 90 equispaced times on [0, 100], AAA poles of exp(-x) on [0, 100 rho(L)]
    (tolerance 1e-13), COCG shifted solves to 1e-6 (on the symmetrised system, one
    sparse product per iteration), FP32 vectors with FP64 coefficients.  One step = one wl_return_prob call (spectral radius estimate, poles,
    rational Krylov basis, projection and the 90 estimates)."""
    import numpy as np
    import torch

    import paper_2601_11338_amd as wl
    import synth

    M, t_max, nt = 30, 100.0, 90
    ts = np.linspace(0.0, t_max, nt)
    log("generating the road-network stand-in")
    rp, ci = synth.road_grid(1400, 1400, 0.7, seed=7)
    n, nnz = len(rp) - 1, int(ci.size)
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    for w_ in (64, 32, 1):  # 16-column groups of the padded 30-column blocks
        g.autotune(torch.float32, w_)
    rhoZ = g.spectral_radius(1.0)
    alpha = 1.0 / (1.0 + rhoZ)
    # reorth 0 as in the default workload (the projection's products)
    op = wl.Operator(g, 1.0, "res", alpha, dtype=torch.float32, tol=1e-7, rho_hint=rhoZ, reorth=0)
    K, _ = op.info()
    log(f"graph n={n} nnz={nnz}; rho(Z_1)={rhoZ:.6f} alpha={alpha:.6f}; Lanczos steps per resolvent product {K}")
    Om = wl.probes(ctx, n, M, seed=2026, law="gauss", dtype=torch.float32)
    op.fdeg()

    def step():
        return op.return_prob(Om, ts, t_max, rho=0.0, pole_time=1.0, aaa_tol=1e-13, solve_tol=1e-6, max_iters=1000)

    for _ in range(args.warmup):
        p, e, poles, info = step()
        log(f"warm-up step done: {info}")
    torch.cuda.synchronize()
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts0 = time.perf_counter()
        p, e, poles, info = step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done in {(time.perf_counter() - ts0) * 1e3:.1f} ms: poles {info['npoles']}, "
            f"COCG iterations {info['iters_total']} (max {info['iters_max']}), rho {info['rho']:.4f}, "
            f"p(1)={p[1]:.5f} p(100)={p[-1]:.3e}")
    t1 = time.perf_counter()
    flat = ctx.kernel_stats(1)  # shifted-solve products with A_1(alpha), 64 wide (30 complex columns)
    lan = ctx.kernel_stats(4)   # Lanczos operator products as 16-column groups (projection, 32 wide)
    oth = ctx.kernel_stats(2)   # single-vector products (spectral radius estimate)
    ctx.set_profiling(False)
    ms = (t1 - t0) * 1e3 / args.steps
    # the library's own count of sparse products times the probe columns they act on
    # (padding to 16-column groups not counted)
    edge_vec = info["products"] * float(nnz)
    value = edge_vec / (ms * 1e-3) / 1e9
    kern = []
    for st, what in ((flat, "shifted-solve products with A_1(alpha) (k_spmm, 64 wide)"),
                     (lan, "grouped Lanczos operator products of the projection (k_spmm, 32 wide)")):
        nl, kms_, kby = st
        if nl:
            kern.append({"what": what, "launches": nl, "total_ms": kms_, "avg_launch_us": kms_ / nl * 1e3,
                         "alg_bytes_per_launch": kby / nl, "achieved": kby / (kms_ * 1e-3) / 1e9})
            log(f"{what}: {nl} launches, avg {kms_ / nl * 1e3:.1f} us, {kby / (kms_ * 1e-3) / 1e9:.0f} GB/s "
                f"algorithmic; {kms_ / args.steps:.0f} of {ms:.0f} ms per step")
    dom = max(kern, key=lambda k: k["total_ms"])
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
            "workload": f"average return probability (Alg. 1, rational Krylov + leave-one-out Nystrom) on a "
                        f"road-network stand-in (1400x1400 lattice, edges kept w.p. 0.7) n={n} nnz={nnz}; "
                        f"L_1(res) alpha=1/(1+rho(Z))={alpha:.5f} ({K} Lanczos steps per product); M={M}, "
                        f"{nt} times on [0, {t_max:g}]; AAA tol 1e-13, COCG tol 1e-6 on the symmetrised resolvent "
                        f"system; FP32 vectors, FP64 "
                        f"coefficients",
            "n": n,
            "nnz": nnz,
            "probes": M,
            "times": nt,
            "lanczos_steps": K,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": dom["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["achieved"] / HBM_PEAK_GBS,
            "traffic": traffic_record("k_spmm_w32_arp_road2m", g.shape(torch.float32, 32)[0])
                       if dom["what"].startswith("grouped") else None,
            "kernel": dom["what"],
            "avg_launch_us": dom["avg_launch_us"],
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "other_kernels": [k for k in kern if k is not dom] +
                             [{"what": "single-vector products (spectral radius estimate)", "launches": oth[0],
                               "total_ms": oth[1]}],
        },
        "rational_krylov": {k: info[k] for k in ("npoles", "nblocks", "solves", "iters_total", "iters_max", "rho",
                                                 "aaa_err", "solve_res", "products")},
        "p_hat": {f"{ts[k]:.3g}": [float(p[k]), float(e[k])] for k in (0, 1, 9, 45, nt - 1)},
    }
    if not args.no_reference:
        # the standard Laplacian L = D - A on the same probes and times (the paper's
        # reference in its return-probability figures), outside the timed region
        opL = wl.Operator(g, 0.0, "linear", 1.0, dtype=torch.float32)
        opL.return_prob(Om, ts, t_max, solve_tol=1e-6, max_iters=1000)
        torch.cuda.synchronize()
        tL = time.perf_counter()
        pL, eL, _, infoL = opL.return_prob(Om, ts, t_max, solve_tol=1e-6, max_iters=1000)
        torch.cuda.synchronize()
        msL = (time.perf_counter() - tL) * 1e3
        log(f"standard Laplacian: {msL:.0f} ms, poles {infoL['npoles']}, COCG iterations {infoL['iters_total']}, "
            f"p(1)={pL[1]:.5f} p(100)={pL[-1]:.3e}")
        out["standard_laplacian"] = {
            "ms": msL,
            "rational_krylov": {k: infoL[k] for k in ("npoles", "solves", "iters_total", "iters_max", "rho")},
            "p_hat": {f"{ts[k]:.3g}": [float(pL[k]), float(eL[k])] for k in (0, 1, 9, 45, nt - 1)},
        }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline_arp(rp, ci, n, alpha, K)
    return out


def cpu_baseline_arp(rp, ci, n, alpha, K):
    """The oracle's sparse resolvent product (CG on A_1(alpha), its default tolerance)
    on 8 Gaussian columns, converted at the GPU's accounting (K products per column)."""
    import numpy as np
    from oracle import sparse

    import synth
    A = sparse.adjacency(n, rp, ci)
    X = synth.gaussian_block(n, 8, seed=5)
    t0 = time.perf_counter()
    sparse.phi_res_apply(A, 1.0, alpha, X)
    dt = time.perf_counter() - t0
    ev = K * A.nnz * X.shape[1]
    return {
        "value": ev / dt / 1e9,
        "unit": "GEdge·vec/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"resolvent product (CG, rtol 1e-14) on 8 columns, counted as {K} products per column "
                  f"like the GPU path; scipy.sparse single-threaded FP64, {dt:.1f} s",
    }


def run_arnoldi_ba1m(args):
    """Exponential weights at a large inverse temperature on the BA graph of the
    default workload (n = 1e6, m = 5): mu = 0.5, beta = 60 / rho(Z_mu) (phi V grows like
    e^60, near the top of the FP32 range), phi V for 16
    Rademacher columns (FP32) by block Arnoldi on the 2n linearisation Z (Krylov
    dimension --arnoldi-steps) and, for comparison, by the truncated series at the same
    accuracy; both checked against an FP64 series evaluation.  One step = one Arnoldi
    phi V."""
    import numpy as np
    import torch

    import paper_2601_11338_amd as wl
    import synth

    n, m, b, K = 1_000_000, 5, 16, args.arnoldi_steps
    log("generating Barabasi-Albert graph")
    rp, ci = synth.barabasi_albert(n, m, seed=2026)
    nnz = int(ci.size)
    X_h = synth.rademacher_block(n, b, seed=3, dtype=np.float32)
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    g.autotune(torch.float32, b)
    g.autotune(torch.float64, b)
    mu = 0.5
    rhoZ = g.spectral_radius(mu)
    beta = 60.0 / rhoZ
    X = torch.tensor(X_h, device="cuda")
    ref_op = wl.Operator(g, mu, "exp", beta, dtype=torch.float64, tol=1e-13)
    Kref, _ = ref_op.info()
    log(f"rho(Z)={rhoZ:.4f} beta={beta:.5f}; FP64 reference series degree {Kref}")
    Yref = ref_op.apply_phi(X.double())
    torch.cuda.synchronize()
    series = wl.Operator(g, mu, "exp", beta, dtype=torch.float32, tol=1e-7)
    Ks, _ = series.info()
    arn = wl.Operator(g, mu, "exp", beta, dtype=torch.float32, krylov_dim=K, method="arnoldi")
    Y = torch.empty_like(X)
    Ys = torch.empty_like(X)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            fn()
            torch.cuda.synchronize()
            log(f"step {i + 1}/{steps} done")
        return (time.perf_counter() - t0) * 1e3 / steps

    def err(Yt):
        return float(torch.linalg.norm(Yt.double() - Yref) / torch.linalg.norm(Yref))

    ctx.set_profiling(True)
    ms = timed(lambda: arn.apply_phi(X, out=Y), args.steps)
    rec = ctx.kernel_stats(0)
    ctx.set_profiling(False)
    ms_series = timed(lambda: series.apply_phi(X, out=Ys), max(1, args.steps // 2))
    e_arn, e_ser = err(Y), err(Ys)
    log(f"Arnoldi K={K}: {ms:.1f} ms, rel. error {e_arn:.2e}; series degree {Ks}: {ms_series:.1f} ms, "
        f"rel. error {e_ser:.2e}")
    launches, kms, kbytes = rec
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    edge_vec = (K + 2) * float(nnz) * b   # K products with Z plus the two of the start block
    value = edge_vec / (ms * 1e-3) / 1e9
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
            "workload": f"barabasi-albert n={n} m={m} nnz={nnz}; exponential weights mu={mu} beta=60/rho(Z)="
                        f"{beta:.5f}; phi V, V 16 Rademacher columns, by block Arnoldi on the 2n linearisation "
                        f"(Krylov dimension {K}); FP32 vectors, FP64 coefficients",
            "n": n,
            "nnz": nnz,
            "block": b,
            "krylov_dim": K,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_spmm product with the linearisation (A V_bot + (mu^2 - mu d) V_top, b=16)",
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
        },
        "accuracy": {"arnoldi_rel_error": e_arn, "series_rel_error": e_ser, "reference": f"FP64 series degree {Kref}"},
        "series_comparison": {"degree": Ks, "ms": ms_series},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline_exp_large(rp, ci, n, mu, beta, X_h, Ks)
    return out


def cpu_baseline_exp_large(rp, ci, n, mu, beta, X, K):
    """The oracle's sparse truncated series (FP64) of the GPU series' degree K on 2 of
    the 16 columns; counted as series products x nnz x columns."""
    from oracle import sparse

    A = sparse.adjacency(n, rp, ci)
    t0 = time.perf_counter()
    sparse.phi_exp_apply(A, mu, beta, X[:, :2].astype("float64"), K=K)
    dt = time.perf_counter() - t0
    return {
        "value": K * A.nnz * 2 / dt / 1e9,
        "unit": "GEdge·vec/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"truncated series of degree {K} on 2 of the 16 columns, scipy.sparse single-threaded FP64, "
                  f"{dt:.1f} s",
    }


def run_cv_rmat22(args):
    """Learned control variate.  Operator: mu = 0.5 (theta = 0.5), exponential with
    beta = 1/lambda_max, truncated series (FP32 vectors).  Training: 200 graphs
    (Barabasi-Albert, SBM, power-law configuration model; 2k..20k nodes), up to 1024
    nodes each with exact diag phi from unit blocks through the operator; the network
    learns from the 8 local features, trained by the library's kernels
    (full batch Adam) on the part of diag phi beyond its exact degree-3 series, scaled by
    the degree-4 weight (prediction = base + scale * net).  Evaluation: R-MAT scale 22
    (edge factor 16, a = 0.57,
    b = c = 0.19), exact diagonal on 4096 sampled nodes, ten probe seeds for each
    M in {16, 64, 256}: plain Gaussian Hutchinson, the same probes with the control
    variate, Gaussian BKS, Rademacher Hutchinson, and the low-order surrogate (exact
    diagonal of the degree-3 series, Hutchinson on the remainder) without and with the
    learned control variate.  err = ||d_hat - d|| / ||d - 1|| over the sampled nodes."""
    import numpy as np
    import torch
    from concurrent.futures import ProcessPoolExecutor

    import paper_2601_11338_amd as wl
    import synth

    mu = 0.5
    ctx = wl.Context(0)
    specs = synth.training_specs(200, seed=7)
    log("generating 200 training graphs")
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        csrs = list(ex.map(_gen_spec, specs, chunksize=4))
    rng = np.random.default_rng(5)
    feats, targs = [], []
    t_data = time.perf_counter()
    for rp, ci in csrs:
        g = wl.Graph(ctx, rp, ci)
        beta = 1.0 / g.lambda_max()
        op = wl.Operator(g, mu, "exp", beta, dtype=torch.float32)
        nodes = np.sort(rng.choice(g.n, size=min(1024, g.n), replace=False)).astype(np.int32)
        f = g.features(beta)
        feats.append(f[torch.as_tensor(nodes, device="cuda").long()])
        # target: the part of diag phi beyond its exact degree-3 series, in units of the
        # degree-4 scale (diag phi = base + scale * net(features))
        targs.append(op.surrogate_target(nodes, width=64))
        del op, g
    F = torch.cat(feats).contiguous()
    T = torch.cat(targs).contiguous()
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t_data
    log(f"training set: {F.shape[0]} nodes ({t_data:.1f} s for exact diagonals and features)")
    net = wl.MLP(ctx, synth.glorot_params(MLP_SHAPES, 1))
    t_train = time.perf_counter()
    steps = 2000
    for it in range(steps):
        lr = 3e-3 if it < 1500 else 1e-3
        loss = net.train_step(F, T, lr)
        if it % 500 == 0 or it == steps - 1:
            log(f"train step {it}: mse {loss:.3e} (target variance {float(T.var()):.3e})")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t_train
    log("generating R-MAT scale 22 on the device")
    rp, ci = synth.rmat_device(22, 16, 0.57, 0.19, 0.19, seed=2022)
    g = wl.Graph(ctx, rp, ci, validate=True)
    n, nnz = g.n, g.nnz
    g.autotune(torch.float32, 64)
    beta = 1.0 / g.lambda_max()
    op = wl.Operator(g, mu, "exp", beta, dtype=torch.float32)
    base, scale = op.surrogate_diag()
    ghat = net.predict(g.features(beta), base, scale)
    # evaluation nodes: 8192 uniform and the 256 of largest degree
    deg = (rp[1:] - rp[:-1]).cpu().numpy()
    hubs = np.argsort(-deg, kind="stable")[:256]
    uni = np.random.default_rng(9).choice(n, size=8192, replace=False)
    S = np.unique(np.concatenate([uni, hubs])).astype(np.int32)
    St = torch.as_tensor(S, device="cuda").long()
    # reference diagonal in FP64 (diag phi - 1 is ~1e-5 here: FP32 rounding near 1 would
    # already be a visible part of it), cross-checked on 64 nodes against the oracle
    op64 = wl.Operator(g, mu, "exp", beta, dtype=torch.float64)
    K64 = op64.info()[0]
    d_true = op64.diag_exact(S, width=64).double()
    den = float(torch.linalg.norm(d_true - 1.0))
    log(f"R-MAT n={n} nnz={nnz}; {S.size} evaluation nodes; ||d - 1|| on them {den:.4e}; FP64 degree {K64}")
    xcheck = cross_check_diag(rp, ci, n, mu, beta, K64, uni[:32], hubs[:32], S, d_true.cpu().numpy())
    del op64
    ones = torch.ones(n, dtype=torch.float32, device="cuda")
    ests = {
        "plain_gauss": dict(law="gauss", estimator="hutchinson", cv=None),
        "const1_cv_gauss": dict(law="gauss", estimator="hutchinson", cv=ones),
        "cv_gauss": dict(law="gauss", estimator="hutchinson", cv=ghat),
        "bks_gauss": dict(law="gauss", estimator="bks", cv=None),
        "rademacher": dict(law="rademacher", estimator="hutchinson", cv=None),
        "surrogate_gauss": dict(law="gauss", estimator="surrogate", cv=None),
        "surrogate_cv_gauss": dict(law="gauss", estimator="surrogate", cv=ghat),
        "surrogate_cv_rademacher": dict(law="rademacher", estimator="surrogate", cv=ghat),
    }
    Ms = [16, 64, 256]
    seeds = range(10)
    errs = {k: {} for k in ests}
    t_eval = time.perf_counter()
    for M in Ms:
        for name, kw in ests.items():
            e = []
            for sd in seeds:
                d, _, _ = op.diag_est(M, 1000 + sd, target="phi", **kw)
                e.append(float(torch.linalg.norm(d[St].double() - d_true)) / den)
            errs[name][M] = float(np.mean(e))
            log(f"M={M} {name}: mean err {errs[name][M]:.4e} over {len(e)} seeds")
    torch.cuda.synchronize()
    t_eval = time.perf_counter() - t_eval
    gain = {M: (errs["plain_gauss"][M] / errs["cv_gauss"][M]) ** 2 for M in Ms}
    gain_sur = {M: (errs["plain_gauss"][M] / errs["surrogate_cv_gauss"][M]) ** 2 for M in Ms}
    learned = ["cv_gauss", "surrogate_cv_gauss", "surrogate_cv_rademacher"]
    plain = [k for k in ests if k not in learned]
    best_plain = {M: min(errs[k][M] for k in plain) for M in Ms}
    best_learned = {M: min(errs[k][M] for k in learned) for M in Ms}
    # > 1: the learned control variate beats every estimator without it at that M
    value = float(np.mean([best_plain[M] / best_learned[M] for M in Ms]))
    passed = errs["cv_gauss"][16] <= errs["plain_gauss"][64] and errs["cv_gauss"][64] <= errs["plain_gauss"][256]
    log("error ratio best non-learned / best learned per M: " +
        ", ".join(f"{M}: {best_plain[M] / best_learned[M]:.3f}" for M in Ms))
    cpu = cpu_baseline_cv(rp, ci, n, mu, beta, op.info()[0], S, d_true.cpu().numpy(), den, errs["plain_gauss"][16])
    return {
        "metric": "diag-estimate error vs probes (learned vs plain)",
        "value": value,
        "unit": "error of the best estimator without the network / error of the best with it (mean over M)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": t_eval * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"learned control variate: mu=0.5 exp beta=1/lambda_max; trained on 200 graphs "
                        f"(BA/SBM/CM, 2k..20k nodes, {F.shape[0]} exact diagonals); evaluated on R-MAT "
                        f"scale 22 ef 16 (n={n}, nnz={nnz}) at 4096 sampled nodes, 10 seeds",
            "n": n,
            "nnz": nnz,
            "probes": Ms,
        },
        "errors": errs,
        "best_nonlearned_over_best_learned": {M: best_plain[M] / best_learned[M] for M in Ms},
        "probe_gain_vs_plain_gauss": gain,
        "probe_gain_surrogate_cv_vs_plain_gauss": gain_sur,
        "reference_cross_check": xcheck,
        "cpu_baseline": cpu,
        "pass_cv16_le_plain64_and_cv64_le_plain256": bool(passed),
        "train_seconds": t_train,
        "target_seconds": t_data,
        "eval_seconds": t_eval,
    }


AMG_FRACS = [1e-3, 10 ** (-2.1666666666666665), 10 ** (-1.3333333333333333), 10 ** (-0.5), 0.9, 0.99]


def run_amg_road2m(args):
    """Multigrid-preconditioned CG (Sec. 4.2, 5.3) on the road-network stand-in (the
    1400 x 1400 lattice of arp-road2m, n = 1.96e6): the walk Laplacian of the NBT
    resolvent (mu = 1, eq. deformed) applied to 16 Gaussian columns in FP64, for alpha =
    10^e / rho(Z_1), e in linspace(-3, -0.5, 4) (the paper's grid) and alpha rho(Z_1) =
    0.9, 0.99, CG to the relative residual 1e-9 with one V-cycle of the aggregation
    hierarchy as preconditioner.  Hierarchies are built before the timed region (their
    setup time is reported).  One step = L X for the six alphas.  value counts the
    library's tally of entries x columns over every sparse product (finest level, coarse
    levels, restrictions and prolongations)."""
    import numpy as np
    import torch

    import paper_2601_11338_amd as wl
    import synth

    b = 16
    log("generating the road-network stand-in")
    rp, ci = synth.road_grid(1400, 1400, 0.7, seed=7)
    n, nnz = len(rp) - 1, int(ci.size)
    ctx = wl.Context(0)
    g = wl.Graph(ctx, rp, ci, validate=True)
    g.autotune(torch.float64, b)
    g.autotune(torch.float64, 1)
    rhoZ = g.spectral_radius(1.0)
    ops = []
    for f in AMG_FRACS:
        op = wl.Operator(g, 1.0, "res", f / rhoZ, dtype=torch.float64, method="amg", rho_hint=rhoZ)
        op.fdeg()
        info = op.amg_info()
        log(f"alpha rho = {f:.4g}: levels {info['rows']} (complexity {info['operator_complexity']:.2f}), setup "
            f"{info['setup_ms']:.0f} ms, walk degrees in {info['iterations']} iterations")
        ops.append(op)
    X = wl.probes(ctx, n, b, seed=2026, law="gauss", dtype=torch.float64)
    Y = torch.empty_like(X)
    # one plain product of the same width, for the paper's "a few SpMVs" comparison
    Z = torch.empty_like(X)
    for _ in range(3):
        g.spmm(X, Z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        g.spmm(X, Z)
    torch.cuda.synchronize()
    spmv_ms = (time.perf_counter() - t0) * 1e2

    def step():
        its, per = [], []
        for op in ops:
            ta = time.perf_counter()
            op.apply_L(X, out=Y)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - ta) * 1e3)
            its.append(op.amg_info()["iterations"])
        return its, per

    for _ in range(args.warmup):
        step()
        log("warm-up step done")
    work0 = sum(op.amg_info()["products"] for op in ops)
    ctx.set_profiling(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        its, per = step()
        log(f"step {i + 1}/{args.steps} done: iterations {its}, ms per L X {['%.1f' % x for x in per]}")
    t1 = time.perf_counter()
    launches, kms, kbytes = ctx.kernel_stats(5)
    ctx.set_profiling(False)
    work = sum(op.amg_info()["products"] for op in ops) - work0
    ms = (t1 - t0) * 1e3 / args.steps
    value = work / args.steps / (ms * 1e-3) / 1e9
    avg_ms = kms / max(launches, 1)
    achieved = (kbytes / max(launches, 1)) / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    per_alpha = []
    for f, op, it, pms in zip(AMG_FRACS, ops, its, per):
        info = op.amg_info()
        per_alpha.append({"alpha_rho": f, "iterations": it, "levels": info["rows"],
                          "operator_complexity": info["operator_complexity"], "setup_ms": info["setup_ms"],
                          "ms_per_LX": pms, "spmv_equivalents": pms / spmv_ms})
    log(f"one 16-column FP64 sparse product: {spmv_ms:.3f} ms; L X costs " +
        ", ".join(f"{p['spmv_equivalents']:.1f}" for p in per_alpha) + " of them")
    cpu = None if args.no_cpu_baseline else cpu_baseline_amg(rp, ci, n, rhoZ, per_alpha[3])
    return {
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
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"multigrid-preconditioned CG: road stand-in 1400x1400 lattice p=0.7 (n={n}, nnz={nnz}); "
                        f"L X of the mu=1 resolvent for alpha rho(Z) in {[round(f, 4) for f in AMG_FRACS]}; "
                        f"16 Gaussian columns; CG rel. tol 1e-9; FP64",
            "n": n,
            "nnz": nnz,
            "block": b,
            "rho_Z": rhoZ,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_record("k_spmm_fp64_w16_amg_road2m", g.shape(torch.float64, b)[0]),
            "kernel": "k_spmm<double,2,8,*> finest-level products of the PCG (A_mu p, residual, l1-Jacobi sweep)",
            "avg_launch_us": avg_ms * 1e3,
            "alg_bytes_per_launch": kbytes / max(launches, 1),
        },
        "per_alpha": per_alpha,
        "spmv_ms": spmv_ms,
        "cpu_baseline": cpu,
    }


def cpu_baseline_amg(rp, ci, n, rhoZ, pa):
    """The oracle's hierarchy and PCG (oracle.amg, scipy sparse products, one thread) on
    one column at alpha rho = 10^-0.5; its work counted as the GPU path counts it
    (entries x columns over every sparse product of the iterations)."""
    import numpy as np
    import scipy.sparse as sp
    from oracle import amg, sparse

    A = sp.csr_matrix(sparse.deformed(sparse.adjacency(n, rp, ci), 1.0, pa["alpha_rho"] / rhoZ))
    x = np.random.default_rng(3).standard_normal(n)
    t0 = time.perf_counter()
    levels = amg.hierarchy(A)
    t1 = time.perf_counter()
    _, its = amg.pcg(A, x, levels, tol=1e-9)
    t2 = time.perf_counter()
    log(f"CPU oracle: hierarchy {t1 - t0:.1f} s, PCG {int(its[0])} iterations in {t2 - t1:.1f} s")
    # per iteration: the operator product, per level above the coarsest a residual and a
    # post-smoothing sweep (the pre-smoothing sweep from zero is a scaling) plus the
    # restriction and prolongation, and the coarsest level's remaining sweeps
    # (the finest level counts the graph's nonzeros, its diagonal being applied in the epilogue)
    nz = [lv[0].nnz for lv in levels]
    nz[0] -= n
    pnnz = sum(lv[1].nnz for lv in levels if lv[1] is not None)
    per_it = nz[0] + sum(2 * z for z in nz[:-1]) + 2 * pnnz + 29 * nz[-1]
    return {"value": per_it * int(its[0]) / (t2 - t1) / 1e9, "unit": "GEdge·vec/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle hierarchy ({t1 - t0:.1f} s) and PCG on 1 of 16 columns at alpha rho(Z) = 10^-0.5, "
                      f"{int(its[0])} iterations in {t2 - t1:.1f} s (scipy sparse products, one thread)"}


def _host_csr(rp, ci, n):
    import numpy as np
    import scipy.sparse as sp
    rph = rp.cpu().numpy().astype(np.int64)
    cih = ci.cpu().numpy()
    return sp.csr_matrix((np.ones(cih.size), cih, rph), shape=(n, n))


def cross_check_diag(rp, ci, n, mu, beta, K, uni, hubs, S, d_gpu):
    """diag phi at 32 uniform and 32 top-degree nodes from the oracle's FP64 series
    (unit columns pushed through eq. qrec on the CPU, same degree K) against the GPU's
    FP64 reference diagonal."""
    import numpy as np
    from oracle import krylov

    t0 = time.perf_counter()
    As = _host_csr(rp, ci, n)
    nodes = np.concatenate([uni, hubs]).astype(np.int64)
    E = np.zeros((n, nodes.size))
    E[nodes, np.arange(nodes.size)] = 1.0
    Y = krylov.series_apply(As, mu, krylov.exp_coefficients(beta, K), E)
    d_cpu = Y[nodes, np.arange(nodes.size)]
    pos = np.searchsorted(S, nodes)
    d_g = d_gpu[pos]
    live = d_cpu != 1.0  # isolated nodes have d = 1 exactly: judged by the absolute error alone
    rel = np.abs(d_g - d_cpu)[live] / np.abs(d_cpu - 1.0)[live]
    secs = time.perf_counter() - t0
    worst = float(rel.max()) if rel.size else None
    log(f"reference cross-check on {nodes.size} nodes (32 uniform, 32 hubs; {int((~live).sum())} isolated): "
        f"max |d_gpu - d_cpu| / |d - 1| = {worst} ({secs:.1f} s on {krylov.threads()} threads)")
    return {"nodes": int(nodes.size), "isolated": int((~live).sum()), "max_rel_err_of_d_minus_1": worst,
            "max_abs_err": float(np.abs(d_g - d_cpu).max()), "seconds": secs}


def cpu_baseline_cv(rp, ci, n, mu, beta, K, S, d_true, den, gpu_err):
    """The plain Gaussian estimator at M = 16 (seed 1000) recomputed by the oracle: the
    same Philox probes (oracle.philox), phi Omega by the FP64 series on a row-chunked
    thread pool, Hutchinson's diagonal; its error against the same reference."""
    import numpy as np
    from oracle import estimators, krylov, philox

    As = _host_csr(rp, ci, n)
    t0 = time.perf_counter()
    Om = philox.gaussian(n, 16, 1000)
    Y = krylov.series_apply(As, mu, krylov.exp_coefficients(beta, K), Om)
    d = estimators.hutchinson_diag(Om, Y)
    secs = time.perf_counter() - t0
    err = float(np.linalg.norm(d[S] - d_true) / den)
    log(f"CPU oracle: plain Gaussian M=16 seed 1000 err {err:.4e} (GPU mean over seeds {gpu_err:.4e}), {secs:.1f} s")
    return {"value": K * float(As.nnz) * 16 / secs / 1e9, "unit": "GEdge·vec/s", "cores": krylov.threads(),
            "kind": "oracle",
            "sample": f"plain Gaussian Hutchinson, M = 16 (seed 1000), degree-{K} FP64 series on a row-chunked "
                      f"thread pool, {secs:.1f} s; its error {err:.4e}"}


def run_ba1m_packed(args, rp, ci, n, m, nnz, K, b, X_h, ctx, g):
    """The default workload with every operator group in one wide block: the five
    exponential operators (truncated series) and the five resolvent operators (block
    Lanczos) each evaluate L V of all five and their walk degrees w = f(A)1 together
    (wl_multi_apply_fdeg: 5 x 16 columns plus a 16-column group holding the five
    vectors of ones, 96 FP32 values = three whole cache lines per gathered row).  The
    resolvent group runs on a second stream (its own library context borrowing the
    device CSR) while the series group runs on the first."""
    import threading

    import torch

    import paper_2601_11338_amd as wl

    wd = 5 * b + 16
    if args.shapes:
        for item in args.shapes.split(","):
            w_, l_, t_ = (int(x) for x in item.split(":"))
            g.set_shape(torch.float32, w_, l_, t_)
    else:
        for w_ in (wd, b, 2 * b, 5):
            g.autotune(torch.float32, w_)
    log("launch shapes width:lanes:threshold " +
        ",".join(f"{w_}:{g.shape(torch.float32, w_)[0]}:{g.shape(torch.float32, w_)[1]}" for w_ in (wd, b, 2 * b, 5)))
    lam = g.lambda_max()
    mus = [0.0, 0.25, 0.5, 0.75, 1.0]
    rhos = []
    for mu in mus:
        rhos.append(g.spectral_radius(mu))
        log(f"mu={mu}: rho(Z_mu)={rhos[-1]:.6f} (lambda_max={lam:.6f})")
    X = torch.tensor(X_h, device="cuda")
    exp_ops = [wl.Operator(g, mu, "exp", 1.0 / lam, dtype=torch.float32, krylov_dim=K) for mu in mus]
    series = wl.Multi(exp_ops)
    Ys = torch.empty((n, 5 * b), dtype=torch.float32, device="cuda")
    Ws = torch.empty((n, 5), dtype=torch.float32, device="cuda")
    series.apply_fdeg(X, out=Ys, out_w=Ws)  # walk degrees cached for the Laplacian finish
    packed = args.res_layout == "packed"
    # resolvent work items, each on its own context (stream) borrowing the device CSR
    nitems = 1 if packed else 3
    nctx = min(nitems, max(1, args.streams - 1))
    ctxs, rgraphs = [ctx], []
    for _ in range(nctx):
        if args.streams > 1:
            c = wl.Context(0, stream=torch.cuda.Stream().cuda_stream)
            gi = wl.Graph(c, g.rowptr, g.colidx)
            for w_ in (wd, b, 2 * b, 5):
                gi.set_shape(torch.float32, w_, *g.shape(torch.float32, w_))
            ctxs.append(c)
            rgraphs.append(gi)
        else:
            rgraphs.append(g)
    keep = []

    # reorth 0: the three-term recurrence with the projection against the current block;
    # against the FP64 oracle its FP32 results equal those of the second local pass
    # (reorth 1: 3.3e-7 against 3.5e-7 relative on these operators), which costs a third
    # of the Gram and update traffic of every Lanczos step
    def res_ops_on(graph):
        return [wl.Operator(graph, mu, "res", 0.5 / rho, dtype=torch.float32, krylov_dim=K, rho_hint=rho, reorth=0)
                for mu, rho in zip(mus, rhos)]

    items = []
    if packed:
        resolv = wl.Multi(res_ops_on(rgraphs[0]))
        Yr, Wr = torch.empty_like(Ys), torch.empty_like(Ws)
        resolv.apply_fdeg(X, out=Yr, out_w=Wr)
        keep.append(resolv)
        items.append([lambda: resolv.apply_fdeg(X, out=Yr, out_w=Wr)])
    else:
        per = [[] for _ in rgraphs]
        for i in range(3):  # item i on resolvent context i mod count
            gi = rgraphs[i % len(rgraphs)]
            ops_r = res_ops_on(gi)
            keep.append(ops_r)
            if i == 0:  # L V of the fifth operator with the walk degrees of all five beside it:
                # [16 columns | 5 single-column processes + 11 padding] = one line per row
                fd = wl.Multi(ops_r[4:] + ops_r[:4])
                Wr = torch.empty((n, 5), dtype=torch.float32, device="cuda")
                Y1 = torch.empty((n, b), dtype=torch.float32, device="cuda")
                fd.apply_fdeg(X, nx=1, out=Y1, out_w=Wr)
                keep.extend([fd, Wr, Y1])
                per[i % len(rgraphs)].append(lambda fd=fd, Wr=Wr, Y1=Y1: fd.apply_fdeg(X, nx=1, out=Y1, out_w=Wr))
            else:  # L V of a Lanczos pair (32 wide)
                pm = wl.Multi(ops_r[2 * i - 2:2 * i])
                Yp = torch.empty((n, 2 * b), dtype=torch.float32, device="cuda")
                pm.apply_L(X, out=Yp)
                keep.extend([pm, Yp])
                per[i % len(rgraphs)].append(lambda pm=pm, Yp=Yp: pm.apply_L(X, out=Yp))
        items = per
    torch.cuda.synchronize()
    nstreams = len(ctxs)

    def run_items(its):
        for it in its:
            it()

    def res_item():
        for its in items:
            run_items(its)

    def step():
        if nstreams > 1:
            ths = [threading.Thread(target=run_items, args=(its,)) for its in items]
            for th in ths:
                th.start()
            series.apply_fdeg(X, out=Ys, out_w=Ws)
            for th in ths:
                th.join()
        else:
            series.apply_fdeg(X, out=Ys, out_w=Ws)
            res_item()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for c in ctxs:
        c.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps

    def stats(c, k):
        return c.kernel_stats(k)

    # class 3: the series group's sparse products; class 4: the Lanczos groups' (96 wide
    # packed, or the 32-wide pairs); class 1: a single operator's Lanczos products
    timed = {k: [sum(x) for x in zip(*[stats(c, k) for c in ctxs])] for k in (1, 3, 4)}
    # the kernel roofline from a replay one group at a time on its own stream (with two
    # streams a launch's HIP-event interval also spans the other group's work)
    for c in ctxs:
        c.set_profiling(False)
        c.set_profiling(True)
    for _ in range(2):
        series.apply_fdeg(X, out=Ys, out_w=Ws)
        torch.cuda.synchronize()
        res_item()
        torch.cuda.synchronize()
    kern = []
    lanes = g.shape(torch.float32, wd)[0]
    seg = wd // 4  # 16-byte vectors per row
    lpn = 16 if seg % 16 == 0 else (32 if 16 < seg < 32 and lanes >= 32 else (8 if seg % 8 == 0 else 4))
    res_w = wd if packed else 2 * b
    for k, width, what in ((3, wd, "series steps of the five exponential operators and their walk degrees"),
                           (4, res_w, "Lanczos operator products of the five resolvent operators and their walk "
                                      "degrees" if packed else "Lanczos operator products of two resolvent operators, "
                                      "or of one with the five walk-degree processes"),
                           (1, b, "Lanczos operator products of one resolvent operator")):
        nl, kms, kby = [sum(x) for x in zip(*[stats(c, k) for c in ctxs])]
        if nl == 0:
            continue
        kl = g.shape(torch.float32, width)[0]
        sg = width // 4
        kp = 16 if sg % 16 == 0 else (32 if 16 < sg < 32 and kl >= 32 else (8 if sg % 8 == 0 else 4))
        kern.append({"kernel": f"k_spmm<float,4,{kp},{kl}>", "width": width, "what": what, "launches": nl,
                     "total_ms": kms, "avg_launch_us": kms / nl * 1e3, "alg_bytes_per_launch": kby / nl,
                     "achieved": kby / (kms * 1e-3) / 1e9, "class": k,
                     "timed_region": {"launches": timed[k][0], "avg_launch_us": timed[k][1] / max(timed[k][0], 1) * 1e3,
                                      "achieved": timed[k][2] / (timed[k][1] * 1e-3) / 1e9 if timed[k][1] else None}})
    for c in ctxs:
        c.set_profiling(False)
    edge_vec = 10 * K * nnz * (1 + b)
    value = edge_vec / (ms * 1e-3) / 1e9
    dom = max(kern, key=lambda k: k["total_ms"])
    for k in kern:
        log(f"width {k['width']} ({k['what']}): {k['launches']} launches, avg {k['avg_launch_us']:.1f} us, "
            f"{k['achieved']:.0f} GB/s algorithmic, {k['total_ms']:.1f} ms in the replayed steps")
    # gathered 128-byte lines per launch (every row segment of a neighbour, three whole
    # lines at 96 FP32 values) plus the row-aligned streams: the traffic the measured
    # random-gather ceiling applies to
    line_bytes = nnz * 4 * dom["width"] + (dom["alg_bytes_per_launch"] - 4.0 * n * dom["width"])
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
            "operators": 10,
            "streams": nstreams,
            "series_width": wd,
            "resolvent_layout": args.res_layout,
            "lanczos_reorth": 0,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": dom["achieved"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["achieved"] / HBM_PEAK_GBS,
            "traffic": measured_traffic(n, m, dom["width"], g.shape(torch.float32, dom["width"])[0]),
            "kernel": f"{dom['kernel']} ({dom['width']} wide: {dom['what']})",
            "avg_launch_us": dom["avg_launch_us"],
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "line_bytes_per_launch": line_bytes,
            "line_GBps": line_bytes / (dom["avg_launch_us"] * 1e-6) / 1e9,
            "other_kernels": [k2 for k2 in kern if k2 is not dom],
            "measured_in": "replay of the step one group at a time after the timed region",
        },
    }
    # the dominant kernel gathers rows of width x 4 bytes: the same row size for the probe
    ceil = machine_ceilings(ctx, min(512, 4 * dom["width"]))
    out["roofline"]["measured_ceilings"] = ceil
    out["roofline"]["frac_of_gather_ceiling"] = out["roofline"]["line_GBps"] / ceil["gather_line_GBps"]
    log(f"this box: copy {ceil['copy_GBps']:.0f} GB/s, random {ceil['gather_row_bytes']}-byte row gathers "
        f"{ceil['gather_line_GBps']:.0f} GB/s of 128-byte lines; the dominant kernel moves "
        f"{out['roofline']['line_GBps']:.0f} GB/s of lines ({out['roofline']['frac_of_gather_ceiling']:.2f} of that)")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(rp, ci, n, lam, X_h, K)
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (multi-GPU is design-only)",
              file=sys.stderr)
        sys.exit(2)
    if args.summarize:
        if args.window_ms > 0:
            summarize_window(args.summarize, args.window_ms)
        else:
            summarize(args.summarize, args.last)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gather_ceiling:
        gather_ceiling()
        return
    if args.workload == "batch512":
        print(json.dumps(with_nproc(run_batch512(args))), flush=True)
        return
    if args.workload == "cv-rmat22":
        print(json.dumps(with_nproc(run_cv_rmat22(args))), flush=True)
        return
    if args.workload == "expv-rmat25":
        print(json.dumps(with_nproc(run_expv_rmat25(args))), flush=True)
        return
    if args.workload == "markov-ba1m":
        print(json.dumps(with_nproc(run_markov_ba1m(args))), flush=True)
        return
    if args.workload == "arp-road2m":
        print(json.dumps(with_nproc(run_arp_road2m(args))), flush=True)
        return
    if args.workload == "arnoldi-ba1m":
        print(json.dumps(with_nproc(run_arnoldi_ba1m(args))), flush=True)
        return
    if args.workload == "amg-road2m":
        print(json.dumps(with_nproc(run_amg_road2m(args))), flush=True)
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
    if not (args.separate or args.no_pack):
        run_ba1m_packed(args, rp, ci, n, m, nnz, K, b, X_h, ctx, g)
        return
    widths = [b, 1] if args.separate else [b, 1, 4 * b, 5, 2 * b]  # 4 b: four series operators side by
    if args.shapes:                                                    # side; 5: five walk-degree columns;
        for item in args.shapes.split(","):                            # 2 b: two Lanczos processes
            w_, l_, t_ = (int(x) for x in item.split(":"))
            g.set_shape(torch.float32, w_, l_, t_)
    else:
        for w_ in widths:
            g.autotune(torch.float32, w_)
    log("launch shapes width:lanes:threshold " +
        ",".join(f"{w_}:{g.shape(torch.float32, w_)[0]}:{g.shape(torch.float32, w_)[1]}" for w_ in widths))
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
    exp_ops = [op for _, f, op in ops if f == "exp"]
    res_ops = [op for _, f, op in ops if f == "res"]
    res_specs = [(mu, op.desc.rho_hint) for mu, f, op in ops if f == "res"]
    # Work items of one step.  Series operators: walk degrees of all five in one pass
    # (n x 5), L V for four of them on 64-wide rows (two whole cache lines per gathered
    # row), the fifth alone.  Resolvent operators (block Lanczos): walk degrees of all
    # five as five single-column Lanczos processes side by side, L V of two pairs on
    # 32-wide rows (one whole line per gathered row), the fifth alone.  Without
    # side-by-side evaluation (--separate) every operator runs alone.
    W5 = torch.empty((n, len(exp_ops)), dtype=torch.float32, device="cuda")
    Y4 = torch.empty((n, 4 * b), dtype=torch.float32, device="cuda")

    def res_items(graph, ops_r, sel):
        """Callables (those with index in sel) evaluating the resolvent part of a step
        on graph's context."""
        if ops_r is None:
            ops_r = [wl.Operator(graph, mu, "res", 0.5 / rho, dtype=torch.float32, krylov_dim=K, rho_hint=rho)
                     for mu, rho in res_specs]
        W1 = torch.empty((n, 1), dtype=torch.float32, device="cuda")
        Y1 = torch.empty((n, b), dtype=torch.float32, device="cuda")
        keep.extend([ops_r, W1, Y1])
        if args.separate:
            return [(lambda op=op: (op.apply_phi(ones, out=W1), op.apply_L(X, out=Y1)))
                    for i, op in enumerate(ops_r) if i in sel]
        items = []
        if 0 in sel:
            fdeg_all = wl.Multi(ops_r)
            Wr = torch.empty((n, len(ops_r)), dtype=torch.float32, device="cuda")
            ops_r[4].fdeg()  # cached w for the Laplacian finish
            keep.extend([fdeg_all, Wr])
            items.append(lambda: (fdeg_all.fdeg(out=Wr), ops_r[4].apply_L(X, out=Y1)))
        for i, (lo, hi) in ((1, (0, 2)), (2, (2, 4))):
            if i in sel:
                pm = wl.Multi(ops_r[lo:hi])
                Yp = torch.empty((n, 2 * b), dtype=torch.float32, device="cuda")
                pm.apply_L(X, out=Yp)  # walk degrees of the pair, cached for the finish
                keep.extend([pm, Yp])
                items.append(lambda pm=pm, Yp=Yp: pm.apply_L(X, out=Yp))
        return items

    keep = []
    if not args.separate:
        multi_all = wl.Multi(exp_ops)
        multi4 = wl.Multi(exp_ops[:4])
        multi4.apply_L(X, out=Y4)  # walk degrees of the group, cached

    def series_item():
        if args.separate:
            for op in exp_ops:
                op.apply_phi(ones, out=W)
                op.apply_L(X, out=Y)
            return
        multi_all.fdeg(out=W5)
        multi4.apply_L(X, out=Y4)
        exp_ops[4].apply_L(X, out=Y)

    # extra streams: the resolvent items (block Lanczos: latency-bound small kernels
    # between the sparse products) run on their own contexts and streams, each with a
    # graph handle borrowing the same device CSR and the main handle's tuned launch
    # shapes, so their work overlaps
    nstreams = max(1, args.streams) if not args.separate else 1
    ctxs, workers = [ctx], []
    if nstreams > 1:
        import threading
        nitems = 3 if not args.separate else len(res_ops)
        tstreams = [torch.cuda.Stream() for _ in range(min(nstreams - 1, nitems))]
        wgraphs = []
        for ts in tstreams:
            c = wl.Context(0, stream=ts.cuda_stream)
            gi = wl.Graph(c, g.rowptr, g.colidx)
            for bb in (b, 1, 2 * b, 5):  # one kernel instantiation per width
                gi.set_shape(torch.float32, bb, *g.shape(torch.float32, bb))
            ctxs.append(c)
            wgraphs.append(gi)
        # item i runs on worker i mod count, built on that worker's graph
        for wi, gi in enumerate(wgraphs):
            workers.append(res_items(gi, None, {i for i in range(nitems) if i % len(wgraphs) == wi}))
        torch.cuda.synchronize()
        res_serial = None
    else:
        res_serial = res_items(g, res_ops, set(range(len(res_ops))))

    def run_worker(items):
        # the library enqueues on the worker context's stream; the host thread only waits
        # for that stream when a Lanczos run reads its projected matrices
        for it in items:
            it()

    def step():
        if workers:
            threads = [threading.Thread(target=run_worker, args=(wk,)) for wk in workers]
            for t in threads:
                t.start()
        series_item()
        if workers:
            for t in threads:
                t.join()
            return
        run_worker(res_serial)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for c in ctxs:
        c.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        torch.cuda.synchronize()
        log(f"step {i + 1}/{args.steps} done")
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps

    def stats(k):
        tot = [0, 0.0, 0.0]
        for c in ctxs:
            st = c.kernel_stats(k)
            tot = [tot[0] + st[0], tot[1] + st[1], tot[2] + st[2]]
        return tot
    # per-width kernel statistics of the timed region itself (events on each launch's
    # stream; with several streams an interval also spans other streams' work)
    timed_kern = {}
    for width, classes in ((b, (0, 1)), (4 * b, (3,)), (2 * b, (4,))):
        st = [stats(k) for k in classes]
        nl, kms, kby = sum(x[0] for x in st), sum(x[1] for x in st), sum(x[2] for x in st)
        if nl:
            timed_kern[width] = {"launches": nl, "avg_launch_us": kms / nl * 1e3,
                                 "achieved": kby / (kms * 1e-3) / 1e9}
    if len(ctxs) > 1:
        # With several streams the kernels of different operators share the memory
        # system, and the HIP events around one launch also span others' work.  The
        # kernel roofline therefore comes from a serialized replay of the same step
        # (same kernels, shapes and data; one stream at a time) right after the timed
        # region; the timed region's own figures are reported beside it.
        for c in ctxs:
            c.set_profiling(False)
            c.set_profiling(True)
        for _ in range(2):
            series_item()
            torch.cuda.synchronize()
            for wk in workers:
                run_worker(wk)
                torch.cuda.synchronize()
        roofline_phase = "serialized replay of the step after the concurrent timed region"
    else:
        roofline_phase = "timed region"
    # sparse-product kernels by width: the 16-wide product (one instantiation serves the
    # series steps of a single operator, class 0, and the Lanczos operator products,
    # class 1), 64-wide side-by-side series steps (class 3), 32-wide side-by-side
    # Lanczos operator products (class 4)
    kern = []
    for width, classes, what in ((b, (0, 1), "series steps and Lanczos operator products of single operators"),
                                 (4 * b, (3,), "four series operators side by side"),
                                 (2 * b, (4,), "two Lanczos operator products side by side")):
        st = [stats(k) for k in classes]
        nl, kms, kby = sum(x[0] for x in st), sum(x[1] for x in st), sum(x[2] for x in st)
        if nl == 0:
            continue
        lanes = g.shape(torch.float32, width)[0]
        lpn = min(16, width // 4)
        kern.append({"kernel": f"k_spmm<float,4,{lpn},{lanes}>", "width": width, "what": what, "launches": nl,
                     "total_ms": kms, "avg_launch_us": kms / nl * 1e3, "alg_bytes_per_launch": kby / nl,
                     "achieved": kby / (kms * 1e-3) / 1e9, "lanes": lanes})
    for c in ctxs:
        c.set_profiling(False)
    edge_vec = len(ops) * K * nnz * (1 + b)
    value = edge_vec / (ms * 1e-3) / 1e9
    dom = max(kern, key=lambda k: k["total_ms"])
    for k in kern:
        log(f"width {k['width']} ({k['what']}): {k['launches']} launches, avg {k['avg_launch_us']:.1f} us, "
            f"{k['achieved']:.0f} GB/s algorithmic, {k['total_ms']:.1f} ms in the measured steps")
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
            "streams": len(ctxs),
        },
        "roofline": {
            "bound": "hbm",
            "achieved": dom["achieved"],
            "peak": 8000.0,
            "unit": "GB/s",
            "frac": dom["achieved"] / 8000.0,
            "traffic": measured_traffic(n, m, dom["width"], dom["lanes"]),
            "kernel": f"{dom['kernel']} ({dom['width']} wide: {dom['what']})",
            "avg_launch_us": dom["avg_launch_us"],
            "alg_bytes_per_launch": dom["alg_bytes_per_launch"],
            "other_kernels": [{k2: v for k2, v in k.items() if k2 != "lanes"} for k in kern if k is not dom],
            "measured_in": roofline_phase,
            "timed_region": timed_kern.get(dom["width"]),
        },
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(rp, ci, n, lam, X_h, K)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
