"""Local node features for the learned control variate, float64 (test infrastructure).

Written from their definitions with dense/sparse matrix algebra: degree d = A 1,
2-walk count S2 = A d, triangles t = diag(A^3) / 2, neighbour-degree mean, root mean
square and maximum, clustering 2t / (d (d - 1)); structural counts are scaled by the
operator parameter s and passed through log1p.  The paper has no learned component;
these features are pinned by hand-derived counts on G_{5,8} (Fig. 1), K4, a diamond,
stars and cycles, and by brute-force enumeration (triangles over node triples,
clustering over neighbour pairs) on random graphs.
"""

import numpy as np
import scipy.sparse as sp


def features(n, rowptr, colidx, s):
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    A = sp.csr_matrix((np.ones(colidx.size), colidx, rowptr), shape=(n, n))
    d = np.asarray(A.sum(axis=1)).ravel()
    S2 = A @ d
    t = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() / 2.0
    sq = A @ (d * d)
    mx = np.zeros(n)
    for i in range(n):
        nb = colidx[rowptr[i]:rowptr[i + 1]]
        if nb.size:
            mx[i] = d[nb].max()
    with np.errstate(invalid="ignore", divide="ignore"):
        mean = np.where(d > 0, S2 / np.maximum(d, 1), 0.0)
        rms = np.where(d > 0, np.sqrt(sq / np.maximum(d, 1)), 0.0)
        cc = np.where(d >= 2, 2 * t / np.maximum(d * (d - 1), 1), 0.0)
    return np.stack([np.log1p(s * d), np.log1p(s * s * d), np.log1p(s ** 3 * 2 * t), np.log1p(s * s * S2),
                     np.log1p(s * mean), np.log1p(s * rms), np.log1p(s * mx), cc], axis=1)


def surrogate_terms(A, mu, kind, param):
    """Exact low-order part of diag phi and the scale of the remainder (dense A):
    base = diag sum_{k<=3} c_k q_k (eq. qrec truncated), scale = c_4 max(1, d^2 + S2)
    with S2 = A d (sum of neighbour degrees)."""
    from .genfun import coefficients, phi_series
    c = coefficients(kind, param, 4)
    base = np.diag(phi_series(A, mu, c[:4])).copy()
    d = A.sum(1)
    scale = c[4] * np.maximum(1.0, d * d + A @ d)
    return base, scale
