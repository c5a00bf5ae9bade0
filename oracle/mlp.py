"""Oracle for the learned warm start: an FP64 numpy MLP (test infrastructure).

The network maps 6 normalised cell features to 100 normalised log10 level
populations: 6 -> 256 -> 256 -> 256 -> 100, SiLU(z) = z * sigmoid(z) after each
hidden layer, linear output, loss = mean squared error over batch and outputs.
Parameters are one flat FP32-ordered vector: W1 [256, 6], b1 [256], W2 [256, 256],
b2, W3 [256, 256], b3, W4 [100, 256], b4 [100] (weights row-major [out, in]).
The MLP is not in the paper; its plain definition is the formula above, and
its gradients are pinned by central finite differences.
"""
import numpy as np

SIZES = [6, 256, 256, 256, 100]


def shapes():
    out = []
    for i in range(4):
        out.append((SIZES[i + 1], SIZES[i]))
        out.append((SIZES[i + 1],))
    return out


N_PARAMS = int(sum(np.prod(s) for s in shapes()))


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for s in shapes():
        n = int(np.prod(s))
        out.append(p[off: off + n].reshape(s))
        off += n
    return out


def init_params(seed=0):
    g = np.random.default_rng(seed)
    parts = []
    for s in shapes():
        if len(s) == 2:
            parts.append(g.standard_normal(s).ravel() * np.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(p, x):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for W, b in ((W1, b1), (W2, b2), (W3, b3)):
        z = a @ W.T + b
        cache.append((a, z))
        a = z * _sig(z)
    y = a @ W4.T + b4
    cache.append((a, None))
    return y, cache


def loss_and_grad(p, x, t):
    """MSE over all outputs and its gradient w.r.t. the flat parameters (FP64)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    y, cache = forward(p, x)
    t = np.asarray(t, dtype=np.float64)
    B, O = y.shape
    r = y - t
    loss = float((r * r).sum() / (B * O))
    dy = 2.0 * r / (B * O)
    a3 = cache[3][0]
    gW4 = dy.T @ a3
    gb4 = dy.sum(0)
    da = dy @ W4
    grads = [None] * 8
    grads[6], grads[7] = gW4, gb4
    for li, W in ((2, W3), (1, W2), (0, W1)):
        a_in, z = cache[li]
        s = _sig(z)
        dz = da * (s * (1.0 + z * (1.0 - s)))
        grads[2 * li] = dz.T @ a_in
        grads[2 * li + 1] = dz.sum(0)
        da = dz @ W
    return loss, np.concatenate([g.ravel() for g in grads])


def round_bf16(a):
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
