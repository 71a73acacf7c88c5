"""Benchmark: one Evoformer block forward + backward on one MI355X.

A step is the block forward followed by the block backward (which recomputes
the forward: the block is the activation-checkpoint boundary), on the
initial-training crop N_seq=128, N_res=256, c_m=256, c_z=128, MSA attention
8x32, triangle attention 4x32, triangle-multiplication hidden 128,
outer-product-mean hidden 32, FP32 (the headline workload).  The same block in
BF16 storage with FP32 accumulation is timed beside it.

Prints one JSON line: the FP32 throughput in TFLOP/s of algorithmic work
(value), the BF16 twin, the roofline of the dominant kernel measured with HIP
events around its launches, and the FP64 oracle's throughput on the host.
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
    return inp, flat, w


def step(cfg, dtype, flat, w):
    from paper_2207_05477_amd import binding as B
    B.evoformer_block_fwd(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["mo"], w["zo"], dtype=dtype)
    B.evoformer_block_bwd(cfg, flat, w["m"], w["z"], w["mm"], w["pm"], w["dmo"], w["dzo"], w["dflat"],
                          w["dm"], w["dz"], dtype=dtype)


def time_steps(cfg, dtype, flat, w, steps, warmup):
    for _ in range(warmup):
        step(cfg, dtype, flat, w)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        step(cfg, dtype, flat, w)
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-bf16", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=3)
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    ap.add_argument("--only", choices=["f32", "bf16"], default=None)
    ap.add_argument("--breakdown", action="store_true",
                    help="print a per-(kernel, sub-operation) time breakdown to stderr")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
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

    ms, roof, stats = None, None, []
    if args.only != "bf16":
        inp, flat, w = make_workload(cfg, "f32", dev)
        ms = time_steps(cfg, "f32", flat, w, args.steps, args.warmup)
        print(f"f32 step {ms:.3f} ms", file=sys.stderr, flush=True)
        stats = profile_steps(cfg, "f32", flat, w, args.profile_steps)
        roof = roofline_of(stats, "f32")
        roof["launches_per_step"] = stats[0]["launches"] / args.profile_steps
        roof["traffic"] = recorded_traffic(roof["kernel"], roof["launches_per_step"])
        if args.breakdown:
            print_breakdown(profile_steps(cfg, "f32", flat, w, args.profile_steps, detail=True), "f32",
                            args.profile_steps)
        del w, flat, inp

    bf16 = None
    if not args.no_bf16 and args.only != "f32":
        cfg16 = cfg.replace(dtype="bf16")
        inp, flat, w = make_workload(cfg16, "bf16", dev)
        ms16 = time_steps(cfg16, "bf16", flat, w, args.steps, args.warmup)
        st16 = profile_steps(cfg16, "bf16", flat, w, args.profile_steps)
        r16 = roofline_of(st16, "bf16")
        r16["launches_per_step"] = st16[0]["launches"] / args.profile_steps
        r16["traffic"] = recorded_traffic(r16["kernel"], r16["launches_per_step"])
        if args.breakdown:
            print_breakdown(profile_steps(cfg16, "bf16", flat, w, args.profile_steps, detail=True), "bf16",
                            args.profile_steps)
        print(f"bf16 step {ms16:.3f} ms", file=sys.stderr, flush=True)
        bf16 = {"ms_per_step": ms16, "tflops": flops_step / (ms16 * 1e-3) / 1e12,
                "speedup_vs_f32": (ms / ms16) if ms else None, "roofline": r16,
                "top_kernels": [{k: s[k] for k in ("name", "launches", "total_ms")} for s in st16[:8]]}
        del w, flat, inp

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
                   "opm_hidden": cfg.opm_hidden, "blocks": 1, "algorithmic_gflop_per_step": flops_step / 1e9},
        "roofline": roof,
        "top_kernels": [{k: s[k] for k in ("name", "launches", "total_ms")} for s in stats[:8]],
        "bf16": bf16,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, flops_step)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
