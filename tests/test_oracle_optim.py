"""Pins of the optimizer oracle (oracle/optim.py) against closed forms, brute
force and a library routine (torch.optim.Adam in float64)."""
import math

import torch

from oracle import optim as OO

F64 = torch.float64


def _vec(n, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(n, dtype=F64, generator=g) * scale


def test_global_norm_brute_force():
    g = _vec(37, 1)
    assert math.isclose(OO.global_norm(g), math.sqrt(sum(x * x for x in g.tolist())), rel_tol=1e-14)


def test_clip_below_threshold_is_identity_and_above_hits_max_norm():
    g = _vec(1000, 2)
    n = OO.global_norm(g)
    same, n1 = OO.clip_by_global_norm(g, n * 1.5)
    assert torch.equal(same, g) and n1 == n
    clipped, n2 = OO.clip_by_global_norm(g, n / 4)
    assert n2 == n
    assert math.isclose(OO.global_norm(clipped), n / 4, rel_tol=1e-14)
    # direction kept
    assert torch.allclose(clipped * 4, g, rtol=1e-14, atol=0)


def test_adam_first_step_closed_form():
    g = _vec(100, 3)
    p = _vec(100, 4)
    z = torch.zeros(100, dtype=F64)
    lr, eps = 1e-3, 1e-6
    p1, m1, v1 = OO.adam_step(p, g, z, z, 1, lr, 0.9, 0.999, eps)
    # with zero moments the bias-corrected first step is lr * g / (|g| + eps)
    assert torch.allclose(p1, p - lr * g / (g.abs() + eps), rtol=1e-13, atol=1e-16)
    assert torch.allclose(m1, 0.1 * g, rtol=1e-15, atol=0)
    assert torch.allclose(v1, 0.001 * g * g, rtol=1e-13, atol=0)


def test_adam_matches_torch_optim_adam_over_steps():
    p0 = _vec(257, 5)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-6
    ref = p0.clone().requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)
    for t in range(1, 6):
        g = _vec(257, 10 + t)
        ref.grad = g.clone()
        opt.step()
        p, m, v = OO.adam_step(p, g, m, v, t, lr, b1, b2, eps)
    assert torch.allclose(p, ref.detach(), rtol=1e-12, atol=1e-15)


def test_ema_closed_form_for_constant_parameters():
    e0 = _vec(64, 6)
    p = _vec(64, 7)
    d = 0.999
    e = e0
    for _ in range(10):
        e = OO.ema_update(e, p, d)
    assert torch.allclose(e, p + d ** 10 * (e0 - p), rtol=1e-13, atol=1e-15)
