"""Float64 reference for the learned control variate's network: an MLP
8 -> 64 -> 64 -> 1 with tanh hidden activations, mean-squared-error loss and
Adam updates, with hand-written backpropagation.

The paper has no learned component; this model exists only to predict diag F
for the control-variate estimator.  Parity unpinned by the paper: it is pinned
by finite differences and by torch autograd in float64 (tests).

Parameter vector layout (shared convention with the library, written on each
side independently): W1 (64x8 row-major), b1 (64), W2 (64x64), b2 (64),
W3 (1x64), b3 (1): 4801 values.
Test infrastructure: see the package docstring.
"""

import numpy as np

NIN, NH = 8, 64
SIZES = [(NH, NIN), (NH,), (NH, NH), (NH,), (1, NH), (1,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)


def unpack(p):
    out, o = [], 0
    for s in SIZES:
        k = int(np.prod(s))
        out.append(np.asarray(p[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in parts])


def forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.tanh(X @ W1.T + b1)
    h2 = np.tanh(h1 @ W2.T + b2)
    y = h2 @ W3.T + b3
    return y[:, 0], (h1, h2)


def loss_and_grad(p, X, t):
    """L = mean_i (y_i - t_i)^2 and dL/dp."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    y, (h1, h2) = forward(p, X)
    N = X.shape[0]
    r = y - np.asarray(t, dtype=np.float64)
    L = float(np.mean(r * r))
    dy = (2.0 / N) * r[:, None]
    gW3 = dy.T @ h2
    gb3 = dy.sum(axis=0)
    dz2 = (dy @ W3) * (1.0 - h2 * h2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (1.0 - h1 * h1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return L, pack([gW1, gb1, gW2, gb2, gW3, gb3])


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba); ``step`` counts from 1.  Returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
