"""FP64 reference of the warm-start network -- TEST INFRASTRUCTURE ONLY.

y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with W1 [64][8], W2 [64][64];
parameters flattened as W1, b1, W2, b2, w3, b3 (4801 values).  Loss: mean
squared error over a minibatch.  Backward is the analytic chain rule;
adam_step is Adam (Kingma & Ba, 2015) with bias correction.
"""
import numpy as np

F, H = 8, 64
SIZES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(p, X):
    w = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ w["w3"] + w["b3"][0]
    return y, (X, a1, h1, a2, h2)


def loss_and_grad(p, X, t):
    w = unpack(p)
    y, (X, a1, h1, a2, h2) = forward(p, X)
    b = len(y)
    r = y - np.asarray(t, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / b
    g = {"w3": h2.T @ dy, "b3": np.array([dy.sum()])}
    dh2 = np.outer(dy, w["w3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ w["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return loss, pack(g)


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def features(row_off, col, d=0.85):
    """Warm-start features from their definitions (FP64): log1p(indeg),
    log1p(outdeg), dangling flag, log(n PR_1(v)) = log((1-d) + d (s1(v) +
    n_dangling/n)) with s1(v) = sum_{u->v} 1/outdeg(u), then four zeros."""
    row_off = np.asarray(row_off, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = len(row_off) - 1
    od = np.diff(row_off).astype(np.float64)
    src = np.repeat(np.arange(n), np.diff(row_off))
    indeg = np.bincount(col, minlength=n).astype(np.float64)
    s1 = np.zeros(n)
    np.add.at(s1, col, 1.0 / od[src])
    fd = float((od == 0).sum()) / n
    X = np.zeros((n, F))
    X[:, 0] = np.log1p(indeg)
    X[:, 1] = np.log1p(od)
    X[:, 2] = (od == 0)
    X[:, 3] = np.log((1 - d) + d * (s1 + fd))
    return X
