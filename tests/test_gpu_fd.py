"""Central finite differences of the GPU block forward against the GPU block
backward (FP32), with no oracle gradient involved: for a direction v over the
inputs m, z or one parameter tensor of each sub-operation,

    (L(theta + h v) - L(theta - h v)) / 2h   vs   <grad L, v>,

L = <m_out, dm_out> + <z_out, dz_out> summed in float64 from the GPU outputs.

The inputs are margin-constructed (every ReLU pre-activation at least 0.2 from
zero, far beyond what a step of h = 1e-2 per element moves it), so L is smooth
along each segment.  Error budget of the difference quotient: the rounding of
L, estimated as 10 * ||out_gpu - out_oracle||_2 * rms(d_out) (ten standard
deviations of a sum of independent rounding errors weighted by d_out) divided
by h, plus the truncation error O(h^2) of the central difference, covered by a
relative 1e-3 of |<grad L, v>|.
"""
import pytest
import torch

from oracle import evoformer as O
from synth import make_inputs, round_inputs

from gpu_util import device_view, say, to_dev
from test_gpu_block import SMALL

pytestmark = pytest.mark.gpu

FD_MARGIN = 0.2
H_STEP = 1e-2
REL_TOL = 1e-3
# one parameter tensor per sub-operation (and a LayerNorm gain and a bias)
PARAM_DIRS = [("row_attn", "w_q"), ("row_attn", "w_bias"), ("col_attn", "w_k"), ("msa_trans", "w_1"),
              ("opm", "w_o"), ("tri_mul_out", "w_ap"), ("tri_mul_in", "w_bg"), ("tri_att_start", "w_v"),
              ("tri_att_end", "w_bias"), ("pair_trans", "w_2"), ("row_attn", "ln_z_g"),
              ("tri_mul_out", "b_g")]


@pytest.mark.parametrize("cfg", [SMALL, SMALL.replace(name="small_extra", extra_msa=True, msa_heads=4,
                                                      msa_head_dim=8, msa_input="onehot23")],
                         ids=["evoformer", "extra_msa"])
def test_block_central_difference_f32(cfg):
    from paper_2207_05477_amd import binding as B
    inp = make_inputs(cfg, seed=41, perturb=True)
    inp = round_inputs(O.with_relu_margins(device_view(inp, "f32"), cfg, FD_MARGIN), "f32")
    assert O.relu_margin(inp, cfg) >= 0.99 * FD_MARGIN
    flat = B.FlatParams(inp["params"][0], "cuda")
    base = flat.buffer.clone()
    m, z = to_dev(inp["m"]), to_dev(inp["z"])
    mm, pm = inp["msa_mask"].float().cuda(), inp["pair_mask"].float().cuda()
    dmo64, dzo64 = inp["dm_out"], inp["dz_out"]

    def fwd(m_, z_, buf):
        flat.buffer = buf
        mo, zo = B.evoformer_block_fwd(cfg, flat, m_, z_, mm, pm)
        torch.cuda.synchronize()
        return mo.double().cpu(), zo.double().cpu()

    def loss(m_, z_, buf):
        mo, zo = fwd(m_, z_, buf)
        return ((mo * dmo64).sum() + (zo * dzo64).sum()).item()

    flat.buffer = base
    dm, dz, dflat = B.evoformer_block_bwd(cfg, flat, m, z, mm, pm, to_dev(dmo64), to_dev(dzo64))
    torch.cuda.synchronize()
    dm, dz, dflat = dm.double().cpu(), dz.double().cpu(), dflat.double().cpu()
    # rounding of L at theta, from the forward's error against the oracle
    mo, zo = fwd(m, z, base)
    mo_ref, zo_ref = O.stack_fwd(inp, cfg)
    err = ((mo - mo_ref).norm() ** 2 + (zo - zo_ref).norm() ** 2).sqrt().item()
    rms = ((dmo64.square().sum() + dzo64.square().sum()) / (dmo64.numel() + dzo64.numel())).sqrt().item()
    noise = 10.0 * err * rms / H_STEP
    say(f"  forward error {err:.3e}; noise bound of the quotient {noise:.3e}")

    gen = torch.Generator().manual_seed(42)
    dirs = []
    vm = torch.randn(m.shape, generator=gen, dtype=torch.float64)
    dirs.append(("m", vm, None, (dm * vm).sum().item()))
    vz = torch.randn(z.shape, generator=gen, dtype=torch.float64)
    dirs.append(("z", vz, None, (dz * vz).sum().item()))
    views_g = flat.views(dflat)
    views_p = flat.views(base.double().cpu())
    for sub, name in PARAM_DIRS:
        p = views_p[sub][name]
        scale = p.square().mean().sqrt().item() or 1.0
        v = torch.randn(p.shape, generator=gen, dtype=torch.float64) * scale
        dirs.append((f"{sub}.{name}", v, (sub, name), (views_g[sub][name] * v).sum().item()))

    worst = 0.0
    for tag, v, pname, an in dirs:
        if pname is None:
            if tag == "m":
                lp = loss(to_dev(inp["m"] + H_STEP * v), z, base)
                lm = loss(to_dev(inp["m"] - H_STEP * v), z, base)
            else:
                lp = loss(m, to_dev(inp["z"] + H_STEP * v), base)
                lm = loss(m, to_dev(inp["z"] - H_STEP * v), base)
        else:
            bp, bm = base.clone(), base.clone()
            flat.views(bp)[pname[0]][pname[1]].add_(H_STEP * v.float().cuda())
            flat.views(bm)[pname[0]][pname[1]].sub_(H_STEP * v.float().cuda())
            lp, lm = loss(m, z, bp), loss(m, z, bm)
        fd = (lp - lm) / (2 * H_STEP)
        tol = REL_TOL * abs(an) + noise
        rel = abs(fd - an) / max(abs(an), 1e-30)
        worst = max(worst, rel)
        say(f"    {tag}: fd {fd:.6e} analytic {an:.6e} rel {rel:.2e} (tol {tol / max(abs(an), 1e-30):.2e})")
        assert abs(fd - an) <= tol, f"{tag}: |fd - analytic| = {abs(fd - an):.3e} > {tol:.3e}"
    flat.buffer = base
    say(f"  worst relative difference {worst:.2e}")
