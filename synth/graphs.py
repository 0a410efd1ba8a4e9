"""Seeded graph generators producing simple undirected graphs as CSR arrays.

Every generator returns ``(rowptr, colidx)``: ``rowptr`` int64 of length n+1,
``colidx`` int32 of length nnz, columns sorted within each row, symmetric
(every undirected edge stored in both directions), no self-loops, no duplicate
entries.  This is the input format of both the oracle and the HIP library.
"""

import numpy as np


# --------------------------------------------------------------------------- CSR
def csr_from_edges(n, u, v):
    """Symmetrise, drop loops, dedupe an undirected edge list into CSR."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    order = np.lexsort((cols, rows))
    rows = rows[order]
    cols = cols[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr, cols.astype(np.int32)


def csr_from_dense(A):
    A = np.asarray(A)
    n = A.shape[0]
    u, v = np.nonzero(np.triu(A, 1))
    return csr_from_edges(n, u, v)


def permute_csr(n, rowptr, colidx, seed):
    """Relabel vertices by a seeded random permutation."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n).astype(np.int64)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    cols = colidx.astype(np.int64)
    pu, pv = perm[rows], perm[cols]
    sel = pu < pv
    return csr_from_edges(n, pu[sel], pv[sel])


# ------------------------------------------------------------------ small graphs
def cycle_graph(n):
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n)


def circulant_graph(n, offsets):
    i = np.arange(n)
    us, vs = [], []
    for o in offsets:
        us.append(i)
        vs.append((i + o) % n)
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def complete_graph(n):
    u, v = np.triu_indices(n, 1)
    return csr_from_edges(n, u, v)


def hypercube_graph(dim):
    n = 1 << dim
    i = np.arange(n)
    us, vs = [], []
    for k in range(dim):
        us.append(i)
        vs.append(i ^ (1 << k))
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def star_graph(leaves):
    n = leaves + 1
    return csr_from_edges(n, np.zeros(leaves, dtype=np.int64), np.arange(1, n))


def toy_g58():
    """The 13-node "trap" graph G_{5,8} of the paper's descriptive example
    (Sec. 5.1, Fig. 1): a 5-node path 1-2-3-4-5 plus 8 leaves on node 3.
    Returned 0-based."""
    edges = [(1, 2), (2, 3), (3, 4), (4, 5)] + [(3, k) for k in range(6, 14)]
    u = np.array([a - 1 for a, _ in edges])
    v = np.array([b - 1 for _, b in edges])
    return csr_from_edges(13, u, v)


# ------------------------------------------------------------------ random graphs
def erdos_renyi_gnm(n, m, seed):
    """G(n, m): m distinct undirected edges drawn uniformly without replacement."""
    rng = np.random.default_rng(seed)
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("m exceeds the number of vertex pairs")
    chosen = np.empty(0, dtype=np.int64)
    while chosen.size < m:
        need = m - chosen.size
        u = rng.integers(0, n, size=2 * need + 16)
        v = rng.integers(0, n, size=2 * need + 16)
        ok = u != v
        lo = np.minimum(u[ok], v[ok])
        hi = np.maximum(u[ok], v[ok])
        key = np.concatenate([chosen, lo * n + hi])
        _, first = np.unique(key, return_index=True)
        chosen = key[np.sort(first)][:m]
    lo = chosen // n
    hi = chosen - lo * n
    return csr_from_edges(n, lo, hi)


def barabasi_albert(n, m, seed):
    """Preferential attachment: a seed clique K_{m+1}, then every new node links to
    m distinct existing nodes chosen with probability proportional to degree
    (uniform draws from the list of edge endpoints)."""
    rng = np.random.default_rng(seed)
    m0 = m + 1
    n_edges = m0 * (m0 - 1) // 2 + m * (n - m0)
    ends = np.empty(2 * n_edges, dtype=np.int64)
    cu, cv = np.triu_indices(m0, 1)
    k = cu.size
    ends[0:2 * k:2] = cu
    ends[1:2 * k:2] = cv
    fill = 2 * k
    batch = 1 << 20
    pool = rng.random(batch)
    pp = 0
    for t in range(m0, n):
        targets = set()
        while len(targets) < m:
            if pp == batch:
                pool = rng.random(batch)
                pp = 0
            targets.add(int(ends[int(pool[pp] * fill)]))
            pp += 1
        tl = sorted(targets)
        ends[fill:fill + 2 * m:2] = t
        ends[fill + 1:fill + 2 * m:2] = tl
        fill += 2 * m
    return csr_from_edges(n, ends[0::2], ends[1::2])


def road_grid(nx, ny, p_keep, seed):
    """Road-network stand-in: the nx x ny square lattice (node i * ny + j at row i,
    column j) with every lattice edge kept independently with probability p_keep
    (p_keep = 0.7 gives mean degree 2.8 and maximum degree 4, the planar, nearly
    regular, locally numbered structure of a road map)."""
    rng = np.random.default_rng(seed)
    idx = np.arange(nx * ny, dtype=np.int64).reshape(nx, ny)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    keep = rng.random(u.size) < p_keep
    return csr_from_edges(nx * ny, u[keep], v[keep])


def stochastic_block_model(n, k, mean_degree, ratio, seed):
    """k equal blocks; p_in / p_out = ratio; expected mean degree ``mean_degree``."""
    rng = np.random.default_rng(seed)
    sizes = np.full(k, n // k)
    sizes[: n % k] += 1
    starts = np.concatenate([[0], np.cumsum(sizes)])
    s = n / k
    p_out = mean_degree / (ratio * (s - 1) + (n - s))
    p_in = ratio * p_out
    us, vs = [], []
    for a in range(k):
        for c in range(a, k):
            if a == c:
                pairs = sizes[a] * (sizes[a] - 1) // 2
                p = p_in
            else:
                pairs = sizes[a] * sizes[c]
                p = p_out
            cnt = rng.binomial(pairs, min(p, 1.0))
            if cnt == 0:
                continue
            u = starts[a] + rng.integers(0, sizes[a], size=cnt)
            v = starts[c] + rng.integers(0, sizes[c], size=cnt)
            us.append(u)
            vs.append(v)
    if not us:
        return csr_from_edges(n, [], [])
    return csr_from_edges(n, np.concatenate(us), np.concatenate(vs))


def configuration_model_powerlaw(n, exponent, kmin, kmax, seed):
    """Erased configuration model with P(k) proportional to k^-exponent on [kmin, kmax]."""
    rng = np.random.default_rng(seed)
    ks = np.arange(kmin, kmax + 1)
    p = ks.astype(np.float64) ** (-exponent)
    p /= p.sum()
    deg = rng.choice(ks, size=n, p=p)
    if deg.sum() % 2:
        deg[rng.integers(0, n)] += 1
    stubs = np.repeat(np.arange(n, dtype=np.int64), deg)
    rng.shuffle(stubs)
    return csr_from_edges(n, stubs[0::2], stubs[1::2])


def rmat(scale, edge_factor, a, b, c, seed, chunk=1 << 24):
    """R-MAT (recursive matrix) generator: edge_factor * 2^scale edge draws, each
    choosing one quadrant per level with probabilities (a, b, c, 1-a-b-c);
    symmetrised, deduped, loops dropped, vertices relabelled by a seeded
    permutation."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    keys = []
    ab = a + b
    abc = a + b + c
    for start in range(0, m, chunk):
        cnt = min(chunk, m - start)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for lev in range(scale):
            r = rng.random(cnt)
            bit = np.int64(1) << (scale - 1 - lev)
            down = r >= ab
            right = ((r >= a) & (r < ab)) | (r >= abc)
            u += down * bit
            v += right * bit
        ok = u != v
        lo = np.minimum(u[ok], v[ok])
        hi = np.maximum(u[ok], v[ok])
        keys.append(np.unique(lo * n + hi))
    key = np.unique(np.concatenate(keys))
    perm = rng.permutation(n).astype(np.int64)
    lo = key // n
    hi = key - lo * n
    return csr_from_edges(n, perm[lo], perm[hi])


def batch_specs(count, seed, n_min=1000, n_max=200000):
    """Recipes of a many-graph workload: sizes log-uniform on [n_min, n_max];
    even entries a stochastic block model (4..32 equal blocks, p_in/p_out = 20,
    mean degree 10), odd entries an erased power-law configuration model
    (exponent 2.5, degrees 2..sqrt(n)).  Each recipe carries its own seed."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), count)).astype(np.int64)
    specs = []
    for i, n in enumerate(sizes):
        s = int(seed) * 100003 + i
        if i % 2 == 0:
            specs.append(("sbm", int(n), int(rng.integers(4, 33)), s))
        else:
            specs.append(("cm", int(n), max(3, int(np.sqrt(n))), s))
    return specs


def training_specs(count, seed, n_min=2000, n_max=20000):
    """Recipes of small training graphs shaped like the large workloads: sizes
    log-uniform on [n_min, n_max], cycling Barabasi-Albert (m in 3..6), stochastic
    block model and power-law configuration model recipes."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(n_min), np.log(n_max), count)).astype(np.int64)
    specs = []
    for i, n in enumerate(sizes):
        s = int(seed) * 100003 + i
        kind = ("ba", "sbm", "cm")[i % 3]
        if kind == "ba":
            specs.append(("ba", int(n), int(rng.integers(3, 7)), s))
        elif kind == "sbm":
            specs.append(("sbm", int(n), int(rng.integers(4, 33)), s))
        else:
            specs.append(("cm", int(n), max(3, int(np.sqrt(n))), s))
    return specs


def graph_from_spec(spec):
    """CSR of one recipe from batch_specs / training_specs."""
    kind, n, p, s = spec
    if kind == "sbm":
        return stochastic_block_model(n, p, 10, 20, s)
    if kind == "cm":
        return configuration_model_powerlaw(n, 2.5, 2, p, s)
    if kind == "ba":
        return barabasi_albert(n, p, s)
    raise ValueError(f"unknown graph recipe {kind}")


def rmat_device(scale, edge_factor, a, b, c, seed, device="cuda"):
    """R-MAT drawn on a torch device (for graphs too large for host generation in a
    few seconds): same recipe as ``rmat`` (one quadrant per level with probabilities
    a, b, c, 1-a-b-c; symmetrised, deduped, loops dropped, seeded relabelling) from
    torch's generator, so the edges differ from ``rmat`` for the same seed.  Returns
    device int32 (rowptr, colidx)."""
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = 1 << scale
    m = edge_factor * n
    chunk = 1 << 26
    ab, abc = a + b, a + b + c
    keys = []
    for start in range(0, m, chunk):
        cnt = min(chunk, m - start)
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for lev in range(scale):
            r = torch.rand(cnt, generator=gen, device=device)
            bit = 1 << (scale - 1 - lev)
            u += (r >= ab).to(torch.int64) * bit
            v += (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64) * bit
        ok = u != v
        lo = torch.minimum(u[ok], v[ok])
        hi = torch.maximum(u[ok], v[ok])
        keys.append(torch.unique(lo * n + hi))
        del u, v, ok, lo, hi
    key = torch.unique(torch.cat(keys))
    del keys
    perm = torch.randperm(n, generator=gen, device=device)
    lo = perm[key // n]
    hi = perm[key % n]
    del key
    src = torch.cat([lo, hi])
    dst = torch.cat([hi, lo])
    del lo, hi
    order = torch.argsort(src * n + dst)
    src = src[order]
    colidx = dst[order].to(torch.int32)
    del dst, order
    counts = torch.bincount(src, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    return rowptr.to(torch.int32), colidx
