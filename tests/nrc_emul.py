"""A CPU emulation of the cache's training-step arithmetic on the matrix
cores (test helper; not the oracle).  The oracle computes the relative-L2
gradient of the MLP in FP64; the kernels round to bf16 at fixed points:
every hidden activation as it is stored (after the ReLU), the loss gradient
dL/dy, and every back-propagated error; products of bf16 values are exact
and sums are taken in float32 on the matrix cores (FP64 here).  With
`rounding=False` this is the plain FP64 computation, which the CPU tests pin
to the oracle's gradient."""
from __future__ import annotations

import numpy as np

LAYERS = [(64, 96), (64, 64), (64, 64), (64, 64), (3, 64)]  # (n_out, n_in)


def bf16(x):
    import torch
    return torch.tensor(np.asarray(x, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def split(W):
    out, off = [], 0
    for (o, i) in LAYERS:
        out.append(np.asarray(W[off:off + o * i], np.float64).reshape(o, i))
        off += o * i
    return out


def train_grad(W, feat, target, rounding=True):
    """(loss, gradient [P]) of mean over records and channels of
    (y - t)^2 / (y^2 + 0.01), the denominator held constant"""
    r = bf16 if rounding else (lambda x: np.asarray(x, np.float64))
    Ws = split(W)
    n = feat.shape[0]
    acts = [r(feat)]
    for l in range(4):
        acts.append(r(np.maximum(acts[-1] @ Ws[l].T, 0.0)))
    y = acts[4] @ Ws[4].T
    t = np.asarray(target, np.float64)
    den = y * y + 0.01
    loss = float(((y - t) ** 2 / den).sum() / (3 * n))
    delta = r(2.0 * (y - t) / den / (3 * n))
    grads = [None] * 5
    for l in range(4, -1, -1):
        grads[l] = delta.T @ acts[l]
        if l > 0:
            delta = r((delta @ Ws[l]) * (acts[l] > 0))
    return loss, np.concatenate([g.ravel() for g in grads])
