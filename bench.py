"""Benchmark: one Evoformer block forward + backward on one MI355X.

A step is the block forward followed by the block backward (which recomputes
the forward: the block is the activation-checkpoint boundary), on the
initial-training crop N_seq=128, N_res=256, c_m=256, c_z=128, MSA attention
8x32, triangle attention 4x32, triangle-multiplication hidden 128,
outer-product-mean hidden 32, FP32 (the headline workload).  The same block in
BF16 storage with FP32 accumulation is timed beside it.

Prints one JSON line: the FP32 throughput in TFLOP/s of algorithmic work
(value), the BF16 twin, the roofline of the dominant kernel measured with HIP
events around its launches, the per-class rooflines (attention forward,
attention backward, triangle contraction: algorithmic FLOPs over their summed
launch times against the MFMA peak of the dtype), mean and median step times
with the forward / backward split, the other crop shapes of the paper's
model-settings table (stack of 4 blocks, extra MSA, fine-tuning stack of 8
blocks, long-chain chunked forward, extra MSA at the fine-tuning crop, template
pair stack), and the FP64 oracle's throughput on the host.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys
import time

import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": 157.3e12, "bf16": 2.5e15}     # dense MFMA peaks of MI355X
HBM_PEAK = 8.0e12


def block_flops(cfg) -> float:
    """Algorithmic forward FLOPs (2 x multiply-adds) of one block."""
    S, R, cm, cz = cfg.n_seq, cfg.n_res, cfg.c_m, cfg.c_z
    hm, dm, ht, dt = cfg.msa_heads, cfg.msa_head_dim, cfg.tri_heads, cfg.tri_head_dim
    ch, co, tf = cfg.tri_mul_hidden, cfg.opm_hidden, cfg.transition_factor
    SR, RR = S * R, R * R
    f = 0.0
    # row attention: q,k,v,g projections, pair bias, logits + context, output
    f += 2 * SR * cm * 4 * hm * dm + 2 * RR * cz * hm + 4 * S * hm * R * R * dm + 2 * SR * hm * dm * cm
    # column attention (or global column attention)
    if cfg.extra_msa:
        f += 2 * SR * cm * (2 * hm * dm + 2 * dm) + 4 * R * hm * S * dm + 2 * SR * hm * dm * cm
    else:
        f += 2 * SR * cm * 4 * hm * dm + 4 * R * hm * S * S * dm + 2 * SR * hm * dm * cm
    f += 2 * SR * cm * tf * cm * 2                                   # MSA transition
    f += 2 * SR * cm * 2 * co + 2 * RR * S * co * co + 2 * RR * co * co * cz   # outer product mean
    f += 2 * (2 * RR * cz * (4 * ch + cz) + 2 * ch * R * R * R + 2 * RR * ch * cz)  # tri-mul x2
    f += 2 * (2 * RR * cz * (4 * ht * dt + ht) + 4 * R * ht * R * R * dt + 2 * RR * ht * dt * cz)  # tri-attn x2
    f += 2 * RR * cz * tf * cz * 2                                   # pair transition
    return float(f)


def template_block_flops(cfg) -> float:
    """Algorithmic forward FLOPs of one template pair stack block on one template."""
    R, cz = cfg.n_res, cfg.c_z
    ht, dt, ch, tf = cfg.tri_heads, cfg.tri_head_dim, cfg.tri_mul_hidden, cfg.transition_factor
    RR = R * R
    f = 2 * (2 * RR * cz * (4 * ch + cz) + 2 * ch * R * R * R + 2 * RR * ch * cz)
    f += 2 * (2 * RR * cz * (4 * ht * dt + ht) + 4 * R * ht * R * R * dt + 2 * RR * ht * dt * cz)
    f += 2 * RR * cz * tf * cz * 2
    return float(f)


def make_workload(cfg, dtype, device):
    import synth
    from paper_2207_05477_amd import binding as B
    inp = synth.round_inputs(synth.make_inputs(cfg.replace(n_blocks=1)), dtype)
    dt = B.act_dtype(dtype)
    flat = B.FlatParams(inp["params"][0], device)
    w = {
        "m": inp["m"].to(device=device, dtype=dt).contiguous(),
        "z": inp["z"].to(device=device, dtype=dt).contiguous(),
        "mm": inp["msa_mask"].float().to(device).contiguous(),
        "pm": inp["pair_mask"].float().to(device).contiguous(),
        "dmo": inp["dm_out"].to(device=device, dtype=dt).contiguous(),
        "dzo": inp["dz_out"].to(device=device, dtype=dt).contiguous(),
    }
    w["dflat"] = flat.zeros_like()
    w["mo"], w["zo"] = torch.empty_like(w["m"]), torch.empty_like(w["z"])
    w["dm"], w["dz"] = torch.empty_like(w["m"]), torch.empty_like(w["z"])
    w["saved"] = torch.empty(B.evoformer_block_saved_bytes(cfg, dtype), dtype=torch.uint8, device=device)
    return inp, flat, w


# One step = the block forward + the block backward on one batch.  Default: the
# forward keeps the block's intermediates (a few GB at this shape) and the
# backward consumes them; checkpoint=True: the forward keeps nothing and the
# backward recomputes it (the form a deep stack uses; one more forward).
def fwd_only(cfg, dtype, flat, w, checkpoint=False):
    from paper_2207_05477_amd import binding as B
    if checkpoint:
        B.evoformer_block_fwd(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["mo"], w["zo"], dtype=dtype)
    else:
        B.evoformer_block_fwd_save(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["mo"], w["zo"], w["saved"],
                                   dtype=dtype)


def bwd_only(cfg, dtype, flat, w, checkpoint=False):
    from paper_2207_05477_amd import binding as B
    if checkpoint:
        B.evoformer_block_bwd(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["dmo"], w["dzo"], w["dflat"],
                              w["dm"], w["dz"], dtype=dtype)
    else:
        B.evoformer_block_bwd_saved(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["saved"], w["dmo"], w["dzo"],
                                    w["dflat"], w["dm"], w["dz"], dtype=dtype)


def step(cfg, dtype, flat, w, checkpoint=False):
    fwd_only(cfg, dtype, flat, w, checkpoint)
    bwd_only(cfg, dtype, flat, w, checkpoint)


def timed(fn, steps, warmup):
    """Per-call HIP-event times (ms) of `steps` calls after `warmup` untimed ones:
    (total-window mean, median of the per-call events)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for i in range(steps):
        fn()
        ev[i + 1].record()
    torch.cuda.synchronize()
    per = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    mean = ev[0].elapsed_time(ev[steps]) / steps
    med = per[steps // 2] if steps % 2 else 0.5 * (per[steps // 2 - 1] + per[steps // 2])
    return mean, med


def time_steps(cfg, dtype, flat, w, steps, warmup):
    return timed(lambda: step(cfg, dtype, flat, w), steps, warmup)[0]


def profile_steps(cfg, dtype, flat, w, steps, detail=False):
    """Per-kernel-instance event timings over `steps` steps (library profiler);
    with `detail`, keyed "kernel@sub-operation"."""
    from paper_2207_05477_amd import _abi as A
    lib = A.load()

    class Stat(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 120), ("launches", ctypes.c_int64),
                    ("total_ms", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]
    lib.evo_profile_begin.restype = None
    lib.evo_profile_end.argtypes = [ctypes.POINTER(Stat), ctypes.c_int32]
    lib.evo_profile_end.restype = ctypes.c_int32
    lib.evo_profile_set_detail.argtypes = [ctypes.c_int32]
    lib.evo_profile_set_detail.restype = None
    torch.cuda.synchronize()
    lib.evo_profile_set_detail(1 if detail else 0)
    lib.evo_profile_begin()
    for _ in range(steps):
        step(cfg, dtype, flat, w)
    recs = (Stat * 1024)()
    n = lib.evo_profile_end(recs, 1024)
    lib.evo_profile_set_detail(0)
    if n < 0:
        raise RuntimeError(lib.evo_last_error().decode())
    out = []
    for r in recs[:n]:
        out.append({"name": r.name.decode(), "launches": int(r.launches), "total_ms": r.total_ms,
                    "flops": r.flops, "bytes": r.bytes})
    out.sort(key=lambda d: -d["total_ms"])
    return out


def roofline_of(stats, dtype):
    """Roofline of the dominant kernel: MFMA-bound when its algorithmic
    intensity (FLOP per algorithmic byte) is above the ridge point of `dtype`,
    else HBM-bound."""
    top = stats[0]
    avg_ms = top["total_ms"] / top["launches"]
    ridge = PEAK[dtype] / HBM_PEAK
    if top["flops"] > 0 and (top["bytes"] <= 0 or top["flops"] / top["bytes"] >= ridge):
        achieved = top["flops"] / (top["total_ms"] * 1e-3) / 1e12
        peak = PEAK[dtype] / 1e12
        return {"kernel": top["name"], "bound": "mfma", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                "avg_launch_ms": avg_ms, "launches_per_step": None}
    achieved = top["bytes"] / (top["total_ms"] * 1e-3) / 1e9
    peak = HBM_PEAK / 1e9
    return {"kernel": top["name"], "bound": "hbm", "achieved": achieved, "peak": peak, "unit": "GB/s",
            "frac": achieved / peak, "traffic": None, "avg_launch_ms": avg_ms, "launches_per_step": None}


def kernel_class(name: str):
    """Kernel class of a detail-mode profiler key "kernel@sub-operation tags"."""
    k, _, tag = name.partition("@")
    if k.startswith("attn_fwd_"):
        return "attention_fwd"
    if k.startswith("attn_bwd_"):
        return "attention_bwd"
    if k.startswith("gemm") and "contract" in tag:
        return "triangle_contraction"
    return None


def class_rooflines(stats, dtype, steps):
    """Per-class algorithmic TFLOP/s (FLOPs of the class's launches over their
    summed event times) and fraction of the dtype's dense MFMA peak."""
    out = {}
    for s in stats:
        c = kernel_class(s["name"])
        if c is None:
            continue
        e = out.setdefault(c, {"launches_per_step": 0.0, "ms_per_step": 0.0, "gflop_per_step": 0.0})
        e["launches_per_step"] += s["launches"] / steps
        e["ms_per_step"] += s["total_ms"] / steps
        e["gflop_per_step"] += s["flops"] / steps / 1e9
    for e in out.values():
        e["tflops"] = e["gflop_per_step"] / e["ms_per_step"] if e["ms_per_step"] > 0 else None
        e["peak_tflops"] = PEAK[dtype] / 1e12
        e["frac"] = e["tflops"] / e["peak_tflops"] if e["tflops"] else None
    return out


def print_breakdown(stats, dtype, steps, file=sys.stderr):
    """Per-(kernel, sub-operation) time per step with each entry's own bound."""
    ridge = PEAK[dtype] / HBM_PEAK
    tot = sum(s["total_ms"] for s in stats) / steps
    print(f"-- {dtype}: {tot:.3f} ms/step in {sum(s['launches'] for s in stats) // steps} launches", file=file)
    for s in stats:
        ms = s["total_ms"] / steps
        sec = s["total_ms"] * 1e-3
        if s["flops"] > 0 and (s["bytes"] <= 0 or s["flops"] / s["bytes"] >= ridge):
            frac = s["flops"] / sec / PEAK[dtype]
            kind = "mfma"
        else:
            frac = s["bytes"] / sec / HBM_PEAK
            kind = "hbm"
        print(f"{ms:8.3f} ms {s['launches'] // steps:4d}x {kind} {100 * frac:5.1f}%  {s['name']}", file=file)


KERNEL_SOURCES = {"gemm_": "gemm.hip", "attn_": "attn.hip", "ln_": "misc.hip", "gattn_": "gattn.hip"}


def kernel_source_hash(kernel_name: str):
    import hashlib
    for prefix, fname in KERNEL_SOURCES.items():
        if kernel_name.startswith(prefix):
            path = os.path.join(ROOT, "paper_2207_05477_amd", "csrc", fname)
            with open(path, "rb") as f:
                return hashlib.sha256(f.read()).hexdigest()[:16]
    return None


def recorded_traffic(kernel_name: str, launches_per_step: float):
    """HBM bytes per launch of `kernel_name` from the committed counter summary
    (profiles/traffic.json, FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of
    known size); None when absent or when the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get("kernels", {}).get(kernel_name)
    if not ent or ent.get("source_sha") != kernel_source_hash(kernel_name):
        return None
    return ent["bytes_per_launch"]


def cpu_baseline(cfg, flops_step):
    """The FP64 oracle (as it stands) on the host cores: one block fwd+bwd of a
    bounded sample of the workload."""
    from oracle import evoformer as O
    import synth
    threads = min(os.cpu_count() or 1, 64)
    torch.set_num_threads(threads)
    inp = synth.round_inputs(synth.make_inputs(cfg.replace(n_blocks=1)), "f32")
    t0 = time.perf_counter()
    O.stack_fwd_bwd(inp, cfg)
    dt = time.perf_counter() - t0
    return {"value": flops_step / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"one full block fwd+bwd at the headline shape ({dt:.1f} s)",
            "ms_per_step": dt * 1e3}


def measure_block(cfg, dtype, dev, steps, warmup, profile_steps_n, breakdown=False):
    """One block fwd+bwd at `cfg` in `dtype`: mean / median step, forward and
    backward alone, the dominant kernel's roofline and the class rooflines."""
    inp, flat, w = make_workload(cfg, dtype, dev)
    flops_step = 3.0 * block_flops(cfg)
    ms, med = timed(lambda: step(cfg, dtype, flat, w), steps, warmup)
    fms, fmed = timed(lambda: fwd_only(cfg, dtype, flat, w), steps, 2)
    bms, bmed = timed(lambda: bwd_only(cfg, dtype, flat, w), steps, 2)
    print(f"{dtype} step {ms:.3f} ms (median {med:.3f}); forward {fms:.3f}, backward {bms:.3f}", file=sys.stderr,
          flush=True)
    cms, cmed = timed(lambda: step(cfg, dtype, flat, w, True), steps, 2)
    cfms, _ = timed(lambda: fwd_only(cfg, dtype, flat, w, True), steps, 2)
    cbms, _ = timed(lambda: bwd_only(cfg, dtype, flat, w, True), steps, 2)
    print(f"{dtype} checkpointed step {cms:.3f} ms (median {cmed:.3f}); forward {cfms:.3f}, backward "
          f"{cbms:.3f} (recomputes the forward)", file=sys.stderr, flush=True)
    stats = profile_steps(cfg, dtype, flat, w, profile_steps_n)
    roof = roofline_of(stats, dtype)
    roof["launches_per_step"] = stats[0]["launches"] / profile_steps_n
    roof["traffic"] = recorded_traffic(roof["kernel"], roof["launches_per_step"])
    detail = profile_steps(cfg, dtype, flat, w, profile_steps_n, detail=True)
    classes = class_rooflines(detail, dtype, profile_steps_n)
    if breakdown:
        print_breakdown(detail, dtype, profile_steps_n)
    res = {"ms_per_step": ms, "ms_per_step_median": med, "tflops": flops_step / (ms * 1e-3) / 1e12,
           "fwd_ms": fms, "fwd_ms_median": fmed, "bwd_ms": bms, "bwd_ms_median": bmed,
           "roofline": roof, "roofline_by_class": classes,
           "saved_state_gib": w["saved"].numel() / 2**30,
           "checkpointed": {"ms_per_step": cms, "ms_per_step_median": cmed, "fwd_ms": cfms, "bwd_ms": cbms,
                            "tflops": flops_step / (cms * 1e-3) / 1e12},
           "top_kernels": [{k: s_[k] for k in ("name", "launches", "total_ms")} for s_ in stats[:8]]}
    del w, flat, inp
    torch.cuda.empty_cache()
    return res


def bench_stack(cfg, dtype, dev, steps, warmup):
    """A stack of cfg.n_blocks blocks: every block's forward, then the backward
    chain (each block's backward recomputes its forward); returns ms per step
    and algorithmic TFLOP/s (3 x forward per block)."""
    import synth
    from paper_2207_05477_amd import binding as B
    inp = synth.round_inputs(synth.make_inputs(cfg), dtype)
    dt = B.act_dtype(dtype)
    flats = [B.FlatParams(p, dev) for p in inp["params"]]
    del inp["params"]
    m = inp["m"].to(device=dev, dtype=dt)
    z = inp["z"].to(device=dev, dtype=dt)
    mm, pm = inp["msa_mask"].float().to(dev), inp["pair_mask"].float().to(dev)
    dmo, dzo = inp["dm_out"].to(device=dev, dtype=dt), inp["dz_out"].to(device=dev, dtype=dt)
    del inp
    acts = [(m, z)] + [(torch.empty_like(m), torch.empty_like(z)) for _ in flats]
    dflats = [f.zeros_like() for f in flats]
    gm, gz = torch.empty_like(m), torch.empty_like(z)

    def one():
        for i, f in enumerate(flats):
            B.evoformer_block_fwd(cfg, f, acts[i][0], acts[i][1], mm, pm, acts[i + 1][0], acts[i + 1][1],
                                  dtype=dtype)
        if not cfg.backward:
            return
        gm.copy_(dmo)
        gz.copy_(dzo)
        for i in reversed(range(len(flats))):
            B.evoformer_block_bwd(cfg, flats[i], acts[i][0], acts[i][1], mm, pm, gm, gz, dflats[i], gm, gz,
                                  dtype=dtype)

    ms, med = timed(one, steps, warmup)
    f = block_flops(cfg) * len(flats) * (3.0 if cfg.backward else 1.0)
    del acts, flats, dflats
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "ms_per_step_median": med, "tflops": f / (ms * 1e-3) / 1e12,
            "algorithmic_gflop_per_step": f / 1e9}


def bench_template(cfg, dtype, dev, steps, warmup):
    """The template pair stack: every template through cfg.n_blocks blocks,
    forward then backward (with recompute)."""
    import synth
    from paper_2207_05477_amd import binding as B
    inp = synth.round_inputs(synth.make_template_inputs(cfg), dtype)
    dt = B.act_dtype(dtype)
    flats = [B.FlatParams(p, dev, subops=B.TEMPLATE_SUBOPS) for p in inp["params"]]
    t = inp["t"].to(device=dev, dtype=dt)
    P = inp["pair_mask"].float().to(dev)
    dto = inp["dt_out"].to(device=dev, dtype=dt)
    T = cfg.n_templ
    acts = [[t[n]] + [torch.empty_like(t[n]) for _ in flats] for n in range(T)]
    dflats = [f.zeros_like() for f in flats]
    g = torch.empty_like(t[0])

    def one():
        for n in range(T):
            for i, f in enumerate(flats):
                B.template_pair_block_fwd(cfg, f, acts[n][i], P[n], acts[n][i + 1], dtype=dtype, template_index=n)
        for n in range(T):
            g.copy_(dto[n])
            for i in reversed(range(len(flats))):
                B.template_pair_block_bwd(cfg, flats[i], acts[n][i], P[n], g, dflats[i], g, dtype=dtype,
                                          template_index=n)

    ms, med = timed(one, steps, warmup)
    f = template_block_flops(cfg) * len(flats) * T * 3.0
    del acts, flats, dflats
    torch.cuda.empty_cache()
    return {"ms_per_step": ms, "ms_per_step_median": med, "tflops": f / (ms * 1e-3) / 1e12,
            "algorithmic_gflop_per_step": f / 1e9}


OTHER_CONFIGS = (
    ("C2", "stack of 4 blocks, N_seq=128, N_res=256, fwd+bwd"),
    ("C3", "extra-MSA block, N_extra=1024, N_res=256, c_e=64, fwd+bwd"),
    ("C4a", "fine-tuning stack of 8 blocks, N_seq=512, N_res=384, fwd+bwd"),
    ("C4b", "long-chain block forward, N_seq=128, N_res=1024, 128-row chunks"),
    ("C5", "extra-MSA block at the fine-tuning crop, N_extra=5120, N_res=384, fwd+bwd"),
    ("T", "template pair stack, 4 templates x 2 blocks, c_t=64, N_res=256, fwd+bwd"),
)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the other crop shapes")
    ap.add_argument("--config-steps", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--only", choices=["f32", "bf16"], default=None)
    ap.add_argument("--breakdown", action="store_true",
                    help="print a per-(kernel, sub-operation) time breakdown to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import synth
    from paper_2207_05477_amd import _abi as A
    A.load()
    dev = torch.device("cuda:0")
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"calibration copy: {src.numel() * 4} bytes read, {dst.numel() * 4} bytes written", file=sys.stderr)
        del src, dst
    cfg = synth.get("C1")
    flops_step = 3.0 * block_flops(cfg)       # forward + backward (2x forward), algorithmic

    f32 = None
    if args.only != "bf16":
        f32 = measure_block(cfg, "f32", dev, args.steps, args.warmup, args.profile_steps, args.breakdown)
    bf16 = None
    if not args.no_bf16 and args.only != "f32":
        bf16 = measure_block(cfg.replace(dtype="bf16"), "bf16", dev, args.steps, args.warmup, args.profile_steps,
                             args.breakdown)
        if f32:
            bf16["speedup_vs_f32"] = f32["ms_per_step"] / bf16["ms_per_step"]
    others = {}
    if not args.no_configs and args.only is None:
        for name, what in OTHER_CONFIGS:
            c = synth.get(name)
            print(f"config {name}: {what}", file=sys.stderr, flush=True)
            if name == "T":
                r = bench_template(c.replace(n_blocks=2), "bf16", dev, args.config_steps, 1)
            else:
                r = bench_stack(c.replace(dtype="bf16"), "bf16", dev, args.config_steps, 1)
            r["workload"] = what
            r["dtype"] = "bf16"
            others[name] = r
            print(f"  {r['ms_per_step']:.2f} ms, {r['tflops']:.1f} TFLOP/s", file=sys.stderr, flush=True)

    ms = f32["ms_per_step"] if f32 else None
    out = {
        "metric": "Evoformer block fwd+bwd ms & TFLOP/s at N_res=256, BF16 vs FP32, % MFMA peak",
        "value": flops_step / (ms * 1e-3) / 1e12 if ms else None,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "evoformer_block_fwd_bwd_initial_crop", "n_seq": cfg.n_seq,
                   "n_res": cfg.n_res, "c_m": cfg.c_m, "c_z": cfg.c_z, "msa_heads": "8x32",
                   "tri_heads": "4x32", "tri_mul_hidden": cfg.tri_mul_hidden,
                   "opm_hidden": cfg.opm_hidden, "blocks": 1, "block_checkpoint": False,
                   "algorithmic_gflop_per_step": flops_step / 1e9},
        "roofline": f32["roofline"] if f32 else None,
    }
    if f32:
        out.update({k: f32[k] for k in ("ms_per_step_median", "fwd_ms", "fwd_ms_median", "bwd_ms", "bwd_ms_median",
                                        "saved_state_gib", "checkpointed", "roofline_by_class", "top_kernels")})
    out["bf16"] = bf16
    out["other_configs"] = others or None
    if not args.no_cpu_baseline and args.only != "bf16":
        out["cpu_baseline"] = cpu_baseline(cfg, flops_step)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
