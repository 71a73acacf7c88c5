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


def bf16_weight_view(inp):
    """inp with every matrix weight w_* rounded to BF16 as the BF16 kernels feed
    them to the matrix cores (the pair-bias projections w_bias stay FP32: they
    are applied in FP32); all other parameters unchanged."""
    out = dict(inp)
    key = "params"
    out[key] = [{s: {k: (v.to(torch.bfloat16).to(F64) if k.startswith("w_") and k != "w_bias" else v)
                     for k, v in blk[s].items()} for s in blk} for blk in inp[key]]
    return out


def check_quant(name, got, ref, ref_q, tol, report=None, floor=0.0, efloor=0.0):
    """Gradient check for small BF16 shapes: the error against the oracle on the
    FP32 parameters, gated at the tolerance plus the effect of the BF16 weight
    quantization alone, ||ref_q - ref|| with ref_q the oracle on the same inputs
    with the matrix weights rounded to BF16 (what an exact implementation that
    multiplies BF16 weights would incur; computed from the oracle alone).  At
    fan-ins of 16-32 channels this effect is a sizeable part of the tolerance;
    both numbers are printed."""
    got64 = got.detach().to("cpu", F64)
    ref64 = ref.detach().to("cpu", F64)
    q64 = ref_q.detach().to("cpu", F64)
    d, dq = got64 - ref64, q64 - ref64
    den = max(ref64.norm().item(), floor, 1e-300)
    eden = max(ref64.abs().max().item(), efloor, 1e-300)
    e, a = d.norm().item() / den, dq.norm().item() / den
    em, am = d.abs().max().item() / eden, dq.abs().max().item() / eden
    etol = ETOL["bf16"] if tol > TOL["f32"] else ETOL["f32"]
    if report is not None:
        report[name] = e
    say(f"    {name}: {e:.3e} (max-norm {em:.3e}); BF16 weight quantization alone {a:.3e} (max-norm {am:.3e})")
    assert torch.isfinite(got.detach().float()).all(), f"{name}: non-finite values"
    assert e <= tol + a, f"{name}: normwise relative error {e:.3e} > {tol:.1e} + {a:.3e}"
    assert em <= etol + am, f"{name}: max-norm relative error {em:.3e} > {etol:.1e} + {am:.3e}"
    return e


def storage_rounding(x, u, dtype):
    """RN(x + u) - (x + u): the rounding a correctly rounded implementation
    incurs when it stores the output x + u of a residual op in `dtype` (all
    float64 on the CPU)."""
    from synth import to_storage
    y = (x + u).detach().to("cpu", F64)
    return to_storage(y, dtype) - y


def check_update(name, out, x, u_ref, dtype, report=None, tol=None):
    """Residual update out - x of an op whose output x + u is stored in `dtype`,
    against the exact update u_ref.  The gate is the tolerance on the update
    plus the storage rounding of the exact output (normwise and max-norm):
        ||(out - x) - u_ref|| <= tol ||u_ref|| + ||RN(x + u_ref) - (x + u_ref)||.
    The second term is what storing any result of this format costs; it is
    computed from the oracle's values alone.  In FP32 it is negligible; in BF16
    it dominates when |u| is small against |x| (an average over many keys, a
    long chain)."""
    tol = TOL[dtype] if tol is None else tol
    etol = ETOL["f32"] if tol <= TOL["f32"] else ETOL["bf16"]
    x64 = x.detach().to("cpu", F64)
    got = out.detach().to("cpu", F64) - x64
    ref = u_ref.detach().to("cpu", F64)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    rho = storage_rounding(x64, ref, dtype)
    d = got - ref
    un, um = max(ref.norm().item(), 1e-300), max(ref.abs().max().item(), 1e-300)
    e, em = d.norm().item() / un, d.abs().max().item() / um
    a, am = rho.norm().item() / un, rho.abs().max().item() / um
    if report is not None:
        report[name] = e
        report.setdefault("_max", {})[name] = em
    say(f"    {name}: {e:.3e} (max-norm {em:.3e}); storage rounding of the exact output {a:.3e} "
        f"(max-norm {am:.3e})")
    assert torch.isfinite(out.detach().float()).all(), f"{name}: non-finite values"
    assert e <= tol + a, f"{name}: normwise relative error {e:.3e} > {tol:.1e} + {a:.3e}"
    assert em <= etol + am, f"{name}: max-norm relative error {em:.3e} > {etol:.1e} + {am:.3e}"
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


def margin_view(inp, cfg, dtype, boundary=None, dropout=None):
    """device_view with every transition's b_1 re-chosen by the oracle so that
    each ReLU pre-activation clears zero by MARGIN[dtype] (W_1 stays as drawn);
    the chosen b_1 are rounded to FP32 like every parameter and the margin is
    asserted again on the rounded inputs.  dropout: the run's (seed, offset)."""
    from oracle import evoformer as O
    from synth import round_inputs
    margin = MARGIN[dtype]
    # constructed with 10 % headroom: rounding the chosen b_1 to FP32 can flip
    # a BF16 rounding of a later block's input in a BF16 stack, which moves
    # that block's pre-activations by about a BF16 ulp of the activations
    inp = round_inputs(O.with_relu_margins(device_view(inp, dtype), cfg, 1.1 * margin, boundary, dropout), dtype)
    got = O.relu_margin(inp, cfg, boundary, dropout)
    assert got >= margin, f"ReLU margin {got:.3e} < {margin:.1e}"
    say(f"  ReLU margin {got:.3e} (requested {margin:.1e})")
    return inp


def template_margin_view(inp, cfg, dtype, dropout=None):
    """margin_view for the template pair stack inputs (synth.make_template_inputs)."""
    from oracle import evoformer as O
    from synth import round_inputs
    margin = MARGIN[dtype]
    inp = round_inputs(O.with_template_relu_margins(device_view(inp, dtype), cfg, 1.1 * margin, dropout), dtype)
    probe = {}
    O.template_stack_fwd(inp, cfg, dropout, probe)
    got = min(probe["min_abs"])
    assert got >= margin, f"ReLU margin {got:.3e} < {margin:.1e}"
    say(f"  ReLU margin {got:.3e} (requested {margin:.1e})")
    return inp
