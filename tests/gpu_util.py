"""Shared helpers of the GPU parity tests (comparison metrics, device copies)."""
from __future__ import annotations

import sys

import torch

F64 = torch.float64
TOL = {"f32": 1e-4, "bf16": 2e-2}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_dtype(name):
    return {"f32": torch.float32, "bf16": torch.bfloat16}[name]


def to_dev(x, dtype="f32"):
    return x.to(dev_dtype(dtype)).cuda().contiguous()


def params_dev(p):
    return {k: v.to(torch.float32).cuda().contiguous() for k, v in p.items()}


def rel_err(got, ref):
    """Normwise relative error ||got - ref||_2 / ||ref||_2 (float64 on the CPU)."""
    got = got.detach().to("cpu", F64)
    ref = ref.detach().to("cpu", F64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    den = ref.norm().item()
    num = (got - ref).norm().item()
    if den == 0.0:
        return num
    return num / den


def check(name, got, ref, tol, report=None, floor=0.0):
    """Normwise relative error against ref; `floor` bounds the denominator from
    below for tensors that are zero by an identity (then the error is relative
    to the magnitude of a sibling quantity without the cancellation)."""
    got64 = got.detach().to("cpu", F64)
    ref64 = ref.detach().to("cpu", F64)
    e = (got64 - ref64).norm().item() / max(ref64.norm().item(), floor, 1e-300)
    if report is not None:
        report[name] = e
    say(f"    {name}: {e:.3e}")
    assert torch.isfinite(got.detach().float()).all(), f"{name}: non-finite values"
    assert e <= tol, f"{name}: normwise relative error {e:.3e} > {tol:.1e}"
    return e


def oracle_grads(fn, inputs: dict, upstream):
    """Gradients of <fn(**inputs), upstream> w.r.t. every float64 leaf in `inputs`
    (nested dicts of tensors allowed)."""
    leaves = {}

    def mk(v, path):
        if isinstance(v, dict):
            return {k: mk(x, path + (k,)) for k, x in v.items()}
        if isinstance(v, torch.Tensor) and v.dtype == F64:
            t = v.detach().clone().requires_grad_(True)
            leaves[path] = t
            return t
        return v
    args = {k: mk(v, (k,)) for k, v in inputs.items()}
    out = fn(**args)
    (out * upstream).sum().backward()
    grads = {}
    for path, t in leaves.items():
        d = grads
        for p in path[:-1]:
            d = d.setdefault(p, {})
        d[path[-1]] = t.grad if t.grad is not None else torch.zeros_like(t)
    return out.detach(), grads


def kink_free(inp):
    """The same inputs with the transitions' W_1 set to zero: every ReLU
    pre-activation is then the bias alone, so every ReLU decision is exact in
    any precision (the block's only discrete decisions).  All other sub-ops keep
    their general parameters."""
    for blk in inp["params"]:
        for sub in ("msa_trans", "pair_trans"):
            blk[sub]["w_1"] = torch.zeros_like(blk[sub]["w_1"])
    return inp


# Coarse gate for gradients of full-parameter blocks: ReLU kinks in the
# transitions flip with the rounding of the block's own forward (any change of
# summation order moves which units sit within rounding of zero), and each flip
# moves whole gradient entries.  The kink-free variants are the parity gate.
KINK_TOL = {"f32": 2e-2, "bf16": 0.15}


def device_view(inp, dtype):
    """Inputs as the implementation in `dtype` computes with them: activations
    and upstream gradients in `dtype`; in BF16 also the matrix-operand weights
    (the kernels multiply BF16 copies of them), parameters otherwise FP32."""
    from synth import round_inputs
    return round_inputs(inp, dtype, weights_dtype="bf16" if dtype == "bf16" else None)
