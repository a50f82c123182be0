"""Binary64 reference for the learned direction proposal's network.

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT (see oracle/__init__.py).

The network maps a 32 x 32 occupancy histogram (1024 inputs) through two
ReLU layers of 512 to 64 direction scores.  ``forward``/``backward`` follow
the definitions of a fully connected layer and its gradient.  With
``emulate=True`` every tensor that the GPU keeps in bfloat16 (inputs, weight
copies, hidden activations, upstream gradients fed to the products) is
rounded to bfloat16 at the same place, so the comparison with the GPU
isolates accumulation order only.
"""
import numpy as np

SIZES = (1024, 512, 512, 64)
N_PARAMS = 512 * 1024 + 512 + 512 * 512 + 512 + 64 * 512 + 64


def bf16(a):
    """Round to the nearest bfloat16 (8 significant bits), ties to even."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)                     # a = m * 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0), e - 8)


def split(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    out = []
    for rows, cols in ((512, 1024), (512, None), (512, 512), (512, None), (64, 512), (64, None)):
        k = rows * (cols or 1)
        t = p[o:o + k]
        out.append(t.reshape(rows, cols) if cols else t)
        o += k
    return out   # W1, b1, W2, b2, W3, b3


def join(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def he_init(seed):
    """He-normal weights, zero biases (float32 values)."""
    r = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((1024, 512), (512, 512), (512, 64)):
        parts.append((r.standard_normal((fan_out, fan_in)) * np.sqrt(2.0 / fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def forward(params, X, emulate=True):
    """Scores [B][64] and the cache for backward."""
    W1, b1, W2, b2, W3, b3 = split(params)
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    X = r(X)
    W1, W2, W3 = r(W1), r(W2), r(W3)
    Z1 = X @ W1.T + b1
    H1 = r(np.maximum(Z1, 0.0))
    Z2 = H1 @ W2.T + b2
    H2 = r(np.maximum(Z2, 0.0))
    S = H2 @ W3.T + b3
    return S, (X, W1, W2, W3, H1, H2)


def backward(cache, dS, emulate=True):
    """Gradient of sum(dS * scores) with respect to every parameter, in the
    parameter layout (float64)."""
    X, W1, W2, W3, H1, H2 = cache
    r = bf16 if emulate else (lambda a: np.asarray(a, np.float64))
    dS = r(dS)
    dW3 = dS.T @ H2
    db3 = dS.sum(0)
    dZ2 = r((dS @ W3) * (H2 > 0))
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(0)
    dZ1 = r((dZ2 @ W2) * (H1 > 0))
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(0)
    return join(dW1, db1, dW2, db2, dW3, db3)


def targets(gain):
    g = np.asarray(gain, np.float64)
    mx = g.max(axis=1, keepdims=True)
    return np.where(mx > 0, g / np.where(mx > 0, mx, 1.0), 0.0)


def loss_and_grad(scores, gain):
    """Mean squared error against gain / max(gain) per set, and d loss / d scores."""
    t = targets(gain)
    d = np.asarray(scores, np.float64) - t
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


def adam(params, grads, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new params, m, v."""
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def top_directions(scores, k=8, gap=0):
    """Indices of the k largest scores per row, largest first, lower index on
    ties (NaN counts as -inf).  With gap > 0 every pick also rules out the
    directions within gap steps of it on the circle of len(row)."""
    s = np.where(np.isnan(scores), -np.inf, np.asarray(scores, np.float64))
    if gap == 0:
        order = np.lexsort((np.broadcast_to(np.arange(s.shape[1]), s.shape), -s), axis=1)
        return order[:, :k]
    D = s.shape[1]
    out = np.zeros((s.shape[0], k), np.int64)
    for r in range(s.shape[0]):
        avail = np.ones(D, bool)
        for j in range(k):
            cand = [d for d in range(D) if avail[d]]
            best = max(cand, key=lambda d: (s[r, d], -d))
            out[r, j] = best
            for d in range(D):
                if min((d - best) % D, (best - d) % D) <= gap:
                    avail[d] = False
    return out
