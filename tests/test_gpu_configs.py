"""Configurations against the FP64 oracle end to end: the FP8 width-512 step
on the 16,384-patch channel, every box of the 32-box batch, the fallback on a
channel box, and a chain of steps in which each step's right-hand side feeds
the next step's residual.

Bars: residual rel-L2 1e-5 (FP32 stencils), correction d and restricted
right-hand side 5e-2 (FP8 network) / 2e-2 (BF16) / 1e-4 (FP32 network over a
three-step chain, fallback sweeps).
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import rel_l2, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2307_14837_amd import batched, stepper

    assert torch.cuda.is_available()
    return batched, stepper


def p32(params):
    return [np.asarray(p, np.float32).astype(np.float64) for p in params]


def test_fp8_width512_step_channel_vs_oracle(mods, orc):
    """One step of the channel 64x16x16 (16,384 patches) with the FP8 network of
    width 512 (the large run's network), indicator evaluated, against the
    oracle's FP64 chain on the same FP32-rounded weights."""
    _, stepper = mods
    w = syn.Workload("chan_fp8", syn.cfg2().box, syn.cfg2().ns, 512, "fp8", "channel")
    say("fp8 width 512 on", w.box.n)
    inp = syn.step_inputs(w, seed=0)
    params = syn.mlp_params(165, 512, 81, seed=0)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="fp8", indicator=True, theta=float("inf"))
    out = st.run_numpy(inp.xc, inp.vprev)
    ref = orc.correction_step(w.box, w.ns, p32(params), inp.xc, out["vprev32"], indicator=True,
                              theta=float("inf"))
    assert rel_l2(out["xt"], ref["xt"]) <= 1e-7
    e = rel_l2(out["r"], ref["r"])
    say(f"  r rel-L2 {e:.2e}")
    assert e <= 1e-5
    for key in ("Y", "d", "bc"):
        e = rel_l2(out[key], ref[key])
        say(f"  {key} rel-L2 {e:.2e}")
        assert e <= 5e-2, key
    say(f"  eta gpu {out['eta']:.6f} oracle {ref['eta']:.6f}")
    assert abs(out["eta"] - ref["eta"]) <= 5e-2 * ref["eta"]


def test_cfg3_every_box_vs_oracle(mods, orc):
    """All 32 uneven periodic boxes of the batched workload, one batched BF16
    step, each box against the oracle (oracle boxes run on host threads)."""
    batched, _ = mods
    boxes = syn.cfg3_boxes(seed=0)
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=6)
    xcs, vps = [], []
    for i, b in enumerate(boxes):
        inp = syn.step_inputs(syn.Workload("b", b, ns, 256, "bf16", "fourier"), seed=20 + i)
        xcs.append(inp.xc)
        vps.append(inp.vprev)
    say(f"cfg3: {len(boxes)} boxes, {sum(b.n_patches for b in boxes)} patches")
    bs = batched.BatchedStep(boxes, ns, params, dtype="bf16")
    bs.load(xcs, vps)
    bs.autotune(reps=2)
    bs.load(xcs, vps)
    bs.step()
    out = bs.results()
    pp = p32(params)

    def ref_of(k):
        vp32 = np.asarray(vps[k], np.float32).astype(np.float64)
        return orc.correction_step(boxes[k], ns, pp, xcs[k], vp32)

    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(ref_of, range(len(boxes))))
    worst = {"d": 0.0, "bc": 0.0, "r": 0.0}
    for k, ref in enumerate(refs):
        d = out[k]["xcorr"][:3].astype(np.float64) - out[k]["xt"][:3]
        ed, eb = rel_l2(d, ref["d"]), rel_l2(out[k]["bc"], ref["bc"])
        ex_ = rel_l2(out[k]["xt"], ref["xt"])
        assert ex_ <= 1e-7, k
        assert ed <= 2e-2 and eb <= 2e-2, (k, boxes[k].n, ed, eb)
        worst["d"], worst["bc"] = max(worst["d"], ed), max(worst["bc"], eb)
    say(f"  worst over boxes: d {worst['d']:.2e}, bc {worst['bc']:.2e}")


def test_fallback_on_channel_box_vs_oracle(mods, orc):
    """The fallback taken (theta = 0) on a channel box of 16x4x4 coarse cells:
    four pressure-held sweeps replace the network's correction, against the
    oracle's sweeps from the same prolongated iterate."""
    _, stepper = mods
    box = syn.channel_box((16, 4, 4))
    w = syn.Workload("chan16", box, syn.NSParams(1e-3, 0.005), 128, "fp32", "channel")
    say("fallback on channel", box.n)
    inp = syn.step_inputs(w, seed=4)
    params = syn.mlp_params(165, 128, 81, seed=4)
    for carry in (True, False):
        st = stepper.CorrectionStep(box, w.ns, params, dtype="fp32", indicator=True, theta=0.0,
                                    fallback_sweeps=4, carry_rhs=carry)
        out = st.run_numpy(inp.xc, inp.vprev)
        ref = orc.correction_step(box, w.ns, p32(params), inp.xc, out["vprev32"], indicator=True, theta=0.0,
                                  fallback_sweeps=4)
        assert out["fell_back"] == ref["fell_back"] == 1
        for key in ("vcorr", "bc"):
            e = rel_l2(out[key], ref[key])
            say(f"  carry_rhs={carry} {key} rel-L2 {e:.2e}")
            assert e <= 1e-4, key
        # the sweeps lowered the momentum residual of x~
        r_fb = orc.residual(box, w.ns, np.concatenate([out["vcorr"], out["xt"][3:4]]), out["vprev32"])
        assert np.linalg.norm(r_fb[:3]) < 0.5 * np.linalg.norm(ref["r"][:3])


def test_three_step_carried_rhs_chain(mods, orc):
    """Three steps in a row on a channel box: step n's right-hand side (built on
    the GPU from its corrected velocity) is the next step's b, and the
    oracle runs the same chain with its own corrected velocity as the next
    v_prev.  Coarse inputs differ per step."""
    _, stepper = mods
    box = syn.channel_box((16, 4, 4))
    w = syn.Workload("chan16", box, syn.NSParams(1e-3, 0.005), 128, "fp32", "channel")
    params = syn.mlp_params(165, 128, 81, seed=9, bias_scale=0.01)
    # small corrections keep the iterates physical over the chain
    params[4] = params[4] * 1e-2
    pp = p32(params)
    ins = [syn.step_inputs(w, seed=30 + n) for n in range(3)]
    st = stepper.CorrectionStep(box, w.ns, params, dtype="fp32")
    assert st.carry_rhs
    vp_gpu0 = np.asarray(ins[0].vprev, np.float32)
    st.load(ins[0].xc, vp_gpu0)
    vprev_ref = vp_gpu0.astype(np.float64)
    for n in range(3):
        say("chain step", n)
        if n > 0:
            st.xc.copy_(torch.as_tensor(np.asarray(ins[n].xc, np.float64).ravel()))
        st.step()
        torch.cuda.synchronize()
        xt = st.xt.cpu().numpy().reshape(4, -1).astype(np.float64)
        r = st.r.cpu().numpy().reshape(4, -1).astype(np.float64)
        vcorr = st.xcorr.cpu().numpy().reshape(4, -1)[:3].astype(np.float64)
        bc = st.bc.cpu().numpy().reshape(4, -1)
        ref = orc.correction_step(box, w.ns, pp, ins[n].xc, vprev_ref)
        er, ev, eb = rel_l2(r, ref["r"]), rel_l2(vcorr - xt[:3], ref["d"]), rel_l2(bc, ref["bc"])
        say(f"  r {er:.2e}  d {ev:.2e}  bc {eb:.2e}")
        assert er <= 1e-5 and ev <= 1e-4 and eb <= 1e-5
        vprev_ref = ref["vcorr"]
