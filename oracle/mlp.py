"""FP64 reference of the warm-start network (TEST INFRASTRUCTURE ONLY: used by tests/, never by the library).

Plain definitions, no blocking or fusion: a 4-layer perceptron x -> tanh(W1 x + b1) -> tanh(W2 . + b2)
-> tanh(W3 . + b3) -> W4 . + b4, the mean squared error over all rows and outputs, its gradient by the
chain rule written out layer by layer, and one bias-corrected Adam step (Kingma & Ba, 2015).  The
parameter vector is laid out as W_l (row-major [out][in]) then b_l for l = 1..4.  When ``bf16`` is set
both operands of every matrix product (weights, layer inputs, back-propagated gradients) are rounded to
bfloat16 (round to nearest even, from their FP32 values), as the GPU path does; the arithmetic stays FP64
and the bias gradients use the unrounded values.  The learned warm start is not part of the paper.
"""

from __future__ import annotations

import numpy as np


def shapes(n_in: int, width: int, n_out: int):
    ins = [n_in, width, width, width]
    outs = [width, width, width, n_out]
    return [(o, i) for i, o in zip(ins, outs)]


def unpack(p: np.ndarray, shp):
    Ws, bs, off = [], [], 0
    for o, i in shp:
        Ws.append(p[off:off + o * i].reshape(o, i))
        off += o * i
        bs.append(p[off:off + o])
        off += o
    assert off == p.size
    return Ws, bs


def pack(Ws, bs) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in zip(Ws, bs)])


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest bfloat16 (ties to even), returned as FP64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _op(a, bf16):
    """Operand of a matrix product as the GPU path feeds it."""
    return round_bf16(a) if bf16 else a


def forward(p, shp, x, bf16=False):
    """Returns the list of layer outputs [a1, a2, a3, y] (a_l = tanh of the pre-activation)."""
    Ws, bs = unpack(np.asarray(p, dtype=np.float64), shp)
    if bf16:
        Ws = [round_bf16(W) for W in Ws]
    a = np.asarray(x, dtype=np.float64)
    outs = []
    for l in range(4):
        z = _op(a, bf16) @ Ws[l].T + bs[l]
        a = np.tanh(z) if l < 3 else z
        outs.append(a)
    return outs


def loss(p, shp, x, t, bf16=False) -> float:
    y = forward(p, shp, x, bf16)[-1]
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def loss_grad(p, shp, x, t, bf16=False):
    """Loss and its gradient with respect to the parameter vector (chain rule, layer by layer)."""
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    Ws, bs = unpack(np.asarray(p, dtype=np.float64), shp)
    if bf16:
        Ws = [round_bf16(W) for W in Ws]
    acts = [x] + forward(p, shp, x, bf16)
    y = acts[-1]
    n = y.size
    L = float(np.sum((y - t) ** 2) / n)
    d = 2.0 * (y - t) / n  # dL/dy
    gW, gb = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        gW[l] = _op(d, bf16).T @ _op(acts[l], bf16)
        gb[l] = d.sum(axis=0)
        if l > 0:
            d = (_op(d, bf16) @ Ws[l]) * (1.0 - acts[l] ** 2)  # through tanh of layer l
    return L, pack(gW, gb)


def adam_step(p, m, v, step, g, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step = 1 for the first); returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
