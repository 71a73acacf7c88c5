"""FP64 CPU oracle of the optimizer step over fused (flat) buffers.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never calls it.  It
shares no code with the HIP path.

The paper fuses every parameter, its gradient and the Adam states (first and
second moments) into a few large tensors (Section "Tensor Fusion") and counts
the kernel launches of three stages on them (the launch-count table of that
section): gradient clipping by global norm (the norm of every gradient
accumulated into one global norm, then every gradient scaled), the Adam update,
and the exponential moving average (EMA) of the parameters.  It takes the
update rules from AlphaFold2 (Section "Hyperparameter setting"); these are the
textbook definitions written out below, on a flat float64 vector.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64


def global_norm(g):
    """Euclidean norm of the whole (fused) gradient: sqrt(sum_i g_i^2)."""
    return math.sqrt(float((g.to(F64) ** 2).sum()))


def clip_by_global_norm(g, max_norm):
    """Scale g by max_norm / max(||g||, max_norm): unchanged when its norm is at
    most max_norm, else rescaled to norm max_norm.  Returns (clipped g, ||g||)."""
    n = global_norm(g)
    scale = max_norm / max(n, max_norm)
    return g.to(F64) * scale, n


def adam_step(p, g, m, v, step, lr, beta1, beta2, eps):
    """One Adam update (step counts from 1):
        m <- beta1 m + (1 - beta1) g
        v <- beta2 v + (1 - beta2) g^2
        p <- p - lr * (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps)
    Returns (p, m, v)."""
    p, g, m, v = (t.to(F64) for t in (p, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (torch.sqrt(vhat) + eps), m, v


def ema_update(e, p, decay):
    """Exponential moving average of the parameters: e <- decay e + (1 - decay) p."""
    return decay * e.to(F64) + (1.0 - decay) * p.to(F64)
