"""CPU reference of the activation proposer's network, loss, optimiser and
block features.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Network 8 -> 64 -> 64 -> 1 with ReLU, ReLU, sigmoid; parameter vector layout
(row-major [in][out]): W1 8x64 @0, b1 @512, W2 64x64 @576, b2 @4672, W3 @4736,
b3 @4800 (4801 values).  Two modes:
  * FP64: the plain definition (used for the finite-difference pin);
  * bf16 emulation: the inputs of every product rounded to bf16 (round to
    nearest even), products accumulated in FP32, as on the GPU's bf16 MFMA.
    The accumulation order of the hardware is not specified, so results agree
    to FP32 rounding, not bit for bit.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NPARAM = 8, 64, 4801
OW1, OB1, OW2, OB2, OW3, OB3 = 0, 512, 576, 4672, 4736, 4800


def unpack(w):
    w = np.asarray(w)
    return (w[OW1:OB1].reshape(8, 64), w[OB1:OW2], w[OW2:OB2].reshape(64, 64), w[OB2:OW3],
            w[OW3:OB3], w[OB3])


def pack(W1, b1, W2, b2, W3, b3, dtype=np.float64):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2), np.ravel(W3),
                           np.atleast_1d(b3)]).astype(dtype)


def bf16(x):
    """Round FP32 values to bf16 (nearest even), returned as FP32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_bits(x):
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation from a seeded PCG64 stream (FP32 master)."""
    r = np.random.default_rng([seed, 7])
    W1 = r.standard_normal((8, 64)) * np.sqrt(2.0 / 8)
    W2 = r.standard_normal((64, 64)) * np.sqrt(2.0 / 64)
    W3 = r.standard_normal(64) * np.sqrt(1.0 / 64)
    return pack(W1, np.zeros(64), W2, np.zeros(64), W3, 0.0, np.float32)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


# ---------------------------------------------------------------------------
# FP64 definition
# ---------------------------------------------------------------------------

def forward64(x, w):
    W1, b1, W2, b2, W3, b3 = (np.asarray(t, np.float64) for t in unpack(w))
    x = np.asarray(x, np.float64)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    z = h2 @ W3 + b3
    return dict(h1=h1, h2=h2, logit=z, prob=sigmoid(z))


def backward64(x, w, fw, dlogit):
    W1, b1, W2, b2, W3, b3 = (np.asarray(t, np.float64) for t in unpack(w))
    x = np.asarray(x, np.float64)
    h1, h2 = fw["h1"], fw["h2"]
    dW3 = h2.T @ dlogit
    db3 = dlogit.sum()
    dh2 = np.outer(dlogit, W3) * (h2 > 0)
    dW2 = h1.T @ dh2
    db2 = dh2.sum(0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    dW1 = x.T @ dh1
    db1 = dh1.sum(0)
    return pack(dW1, db1, dW2, db2, dW3, db3)


def bce(logit, y, pos_weight):
    """Weighted binary cross-entropy on logits, mean over samples; returns
    (loss, dL/dlogit)."""
    z = np.asarray(logit, np.float64)
    y = np.asarray(y, np.float64)
    sp = lambda t: np.logaddexp(0.0, t)  # softplus
    loss = np.mean(pos_weight * y * sp(-z) + (1 - y) * sp(z))
    p = sigmoid(z)
    d = (pos_weight * y * (p - 1) + (1 - y) * p) / z.size
    return loss, d


# ---------------------------------------------------------------------------
# bf16-MFMA emulation
# ---------------------------------------------------------------------------

def forward_bf16(x, w32):
    W1, b1, W2, b2, W3, b3 = (bf16(t) for t in unpack(np.asarray(w32, np.float32)))
    xb = bf16(x)
    h1 = np.maximum((xb @ W1).astype(np.float32) + b1, 0.0).astype(np.float32)
    h2 = np.maximum((bf16(h1) @ W2).astype(np.float32) + b2, 0.0).astype(np.float32)
    z = ((bf16(h2) @ W3).astype(np.float32) + np.float32(b3)).astype(np.float32)
    return dict(h1=h1, h2=h2, logit=z, prob=sigmoid(z.astype(np.float64)))


def backward_bf16(x, w32, fw, dlogit):
    W1, b1, W2, b2, W3, b3 = (bf16(t) for t in unpack(np.asarray(w32, np.float32)))
    dl = np.asarray(dlogit, np.float32)
    h1, h2 = fw["h1"], fw["h2"]
    dW3 = (bf16(h2).T @ bf16(dl)).astype(np.float32)
    db3 = np.float32(dl.sum(dtype=np.float32))
    dh2 = (np.outer(dl, W3) * (h2 > 0)).astype(np.float32)
    dW2 = (bf16(h1).T @ bf16(dh2)).astype(np.float32)
    db2 = dh2.sum(0, dtype=np.float32)
    dh1 = ((bf16(dh2) @ W2.T) * (h1 > 0)).astype(np.float32)
    dW1 = (bf16(x).T @ bf16(dh1)).astype(np.float32)
    db1 = dh1.sum(0, dtype=np.float32)
    return pack(dW1, db1, dW2, db2, dW3, db3, np.float32)


def adam(w, m, v, g, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# block features and labels
# ---------------------------------------------------------------------------

def _signed(i, n):
    i = np.asarray(i)
    return np.where(2 * i < n, i, i - n)


def block_features(dims, block, ab3, G3, mask, eb, step_fraction):
    """Features of every block of one instance (C order over the block grid).

    ab3: three per-block indicator arrays (newest first), G3 their maxima;
    mask: per-block 0/1; eb: per-block energies sum |c_k|^2."""
    nz, ny, nx = dims
    bz, by, bx = block
    gz, gy, gx = nz // bz, ny // by, nx // bx
    nb = gz * gy * gx
    f = np.zeros((nb, 8), np.float64)
    for j in range(3):
        a = np.asarray(ab3[j], np.float64)
        G = float(G3[j])
        with np.errstate(divide="ignore", invalid="ignore"):
            l = np.where((a > 0) & (G > 0), np.log10(np.where(a > 0, a, 1.0) / (G if G > 0 else 1.0)), -40.0)
        f[:, j] = 1.0 + np.clip(l, -40.0, 0.0) / 40.0
    # mean |k| over each block relative to the Nyquist index
    mz = _signed(np.arange(nz), nz).reshape(gz, bz)
    my = _signed(np.arange(ny), ny).reshape(gy, by)
    mx = _signed(np.arange(nx), nx).reshape(gx, bx)
    kk = np.sqrt(mz[:, None, None, :, None, None] ** 2.0 + my[None, :, None, None, :, None] ** 2.0
                 + mx[None, None, :, None, None, :] ** 2.0)
    f[:, 3] = (kk.mean(axis=(3, 4, 5)) / (0.5 * nx)).ravel()
    m = np.asarray(mask).reshape(gz, gy, gx).astype(np.int64)
    act = np.zeros_like(m)
    for ax, g in enumerate((gz, gy, gx)):
        if g < 2:
            continue
        act += np.roll(m, 1, axis=ax) + np.roll(m, -1, axis=ax)
    f[:, 4] = act.ravel() / 6.0
    f[:, 5] = step_fraction
    e = np.asarray(eb, np.float64)
    tot = e.sum()
    with np.errstate(divide="ignore"):
        le = np.where((e > 0) & (tot > 0), np.log10(np.where(e > 0, e, 1.0) * nb / (tot if tot > 0 else 1.0)), -40.0)
    f[:, 6] = np.clip(le, -40.0, 40.0) / 40.0
    f[:, 7] = np.asarray(mask, np.float64)
    return f


def labels(masks):
    """1 where any of the given per-block masks is active."""
    return (np.asarray(masks).reshape(len(masks), -1).max(axis=0) > 0).astype(np.float32)
