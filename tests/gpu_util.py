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


# Element-by-element gate beside the normwise one: max |got - ref| over
# max |ref| of the same tensor.  One wrong element of size |ref| (a masked
# row, a ragged tail tile) moves it to order 1.
ETOL = {"f32": 1e-4, "bf16": 5e-2}


def check(name, got, ref, tol, report=None, floor=0.0, etol=None, efloor=0.0):
    """Normwise relative error ||got - ref||_2 / ||ref||_2 gated at `tol`, and the
    max-norm relative error max|got - ref| / max|ref| gated at `etol` (default:
    the ETOL entry matching `tol`).  `floor` / `efloor` bound the denominators
    from below for tensors that are zero by an identity (then the error is
    relative to the magnitude of a sibling quantity without the cancellation)."""
    got64 = got.detach().to("cpu", F64)
    ref64 = ref.detach().to("cpu", F64)
    assert got64.shape == ref64.shape, (name, got64.shape, ref64.shape)
    d = got64 - ref64
    e = d.norm().item() / max(ref64.norm().item(), floor, 1e-300)
    em = d.abs().max().item() / max(ref64.abs().max().item(), efloor, 1e-300) if d.numel() else 0.0
    if etol is None:
        etol = ETOL["f32"] if tol <= TOL["f32"] else ETOL["bf16"]
    if report is not None:
        report[name] = e
        report.setdefault("_max", {})[name] = em
    say(f"    {name}: {e:.3e} (max-norm {em:.3e})")
    assert torch.isfinite(got.detach().float()).all(), f"{name}: non-finite values"
    assert e <= tol, f"{name}: normwise relative error {e:.3e} > {tol:.1e}"
    assert em <= etol, f"{name}: max-norm relative error {em:.3e} > {etol:.1e}"
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


# ReLU margins of the margin-constructed test inputs (oracle.with_relu_margins):
# far above the pre-activation error of each precision (FP32 about 1e-6, BF16
# about 1e-2 after a stack of blocks), so that every ReLU decision of the
# implementation equals the oracle's.
MARGIN = {"f32": 1e-3, "bf16": 0.1}


def device_view(inp, dtype):
    """Inputs as the implementation in `dtype` receives them at its boundary:
    activations and upstream gradients in `dtype`, parameters FP32 (the FP32
    parameters the ABI takes; the library's own BF16 copies of the weights
    count against it)."""
    from synth import round_inputs
    return round_inputs(inp, dtype)


def margin_view(inp, cfg, dtype, boundary=None):
    """device_view with every transition's b_1 re-chosen by the oracle so that
    each ReLU pre-activation clears zero by MARGIN[dtype] (W_1 stays as drawn);
    the chosen b_1 are rounded to FP32 like every parameter and the margin is
    asserted again on the rounded inputs."""
    from oracle import evoformer as O
    from synth import round_inputs
    margin = MARGIN[dtype]
    inp = round_inputs(O.with_relu_margins(device_view(inp, dtype), cfg, margin, boundary), dtype)
    got = O.relu_margin(inp, cfg, boundary)
    assert got >= 0.99 * margin, f"ReLU margin {got:.3e} < {margin:.1e}"
    say(f"  ReLU margin {got:.3e} (requested {margin:.1e})")
    return inp
