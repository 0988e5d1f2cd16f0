"""Batched multi-box step (plan + fused persistent network stage + autotuner)
against per-box single steps, and HIP-graph replay."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import batched, stepper

    assert torch.cuda.is_available()
    return L, batched, stepper


def batch_inputs(boxes, seed=0):
    xcs, vps = [], []
    for i, b in enumerate(boxes):
        w = syn.Workload("b", b, syn.NSParams(1e-3, 0.01), 256, "bf16", "fourier")
        inp = syn.step_inputs(w, seed=seed + i)
        xcs.append(inp.xc)
        vps.append(inp.vprev)
    return xcs, vps


BOXES = [syn.BoxSpec(n, (1.0, 1.0, 1.0), 7, 0) for n in [(8, 8, 8), (12, 8, 10), (4, 6, 4), (10, 12, 8),
                                                          (6, 4, 2), (16, 8, 12)]]


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8"])
def test_batched_matches_single(mods, dtype):
    L, batched, stepper = mods
    say("batched vs single", dtype)
    ns = syn.NSParams(1e-3, 0.01)
    H = 256
    params = syn.mlp_params(165, H, 81, seed=4)
    xcs, vps = batch_inputs(BOXES)
    bs = batched.BatchedStep(BOXES, ns, params, dtype=dtype)
    bs.load(xcs, vps)
    bs.step()
    out = bs.results()
    for b, box in enumerate(BOXES):
        st = stepper.CorrectionStep(box, ns, params, dtype=dtype)
        ref = st.run_numpy(xcs[b], vps[b])
        assert np.array_equal(out[b]["xt"], ref["xt"].astype(np.float32)), b
        assert np.array_equal(out[b]["Y"], ref["Y"].astype(np.float32)), b
        assert np.array_equal(out[b]["xcorr"][:3], ref["vcorr"].astype(np.float32)), b
        assert np.array_equal(out[b]["bc"], ref["bc"]), b
    # autotuned choice gives the same numbers
    ppt, grid = bs.autotune(reps=3)
    say(f"  autotuned: {ppt} patches per tile, persistent grid {grid}, extension form {bs.plan.scatter_form()}")
    assert ppt in (16, 32, 64)
    assert bs.plan.scatter_form() in (L.SCATTER_NODES, L.SCATTER_TILED)
    bs.load(xcs, vps)  # the step carries the right-hand side: start again
    bs.step()
    out2 = bs.results()
    for b in range(len(BOXES)):
        assert np.array_equal(out2[b]["bc"], out[b]["bc"]), b


MIXED = BOXES[:3] + [syn.BoxSpec((10, 4, 4), (2.5, 0.41, 0.41), 0, 0b110110),  # channel-like, walls
                      syn.BoxSpec((6, 5, 3), (1.0, 1.0, 1.0), 1, 0),
                      syn.BoxSpec((20, 6, 6), (2.0, 1.0, 1.0), 4, 0b000011)]


def test_batched_scatter_forms_agree(mods):
    """The plan's extension stage per node and in tiles: the same sums in the
    same order, so the corrected iterate is bit for bit the same, on periodic,
    partly periodic and walled boxes of uneven sizes (tiles cut by the mesh
    end, periodic axes shorter than a tile)."""
    L, batched, stepper = mods
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=6)
    xcs, vps = batch_inputs(MIXED, seed=20)
    outs = {}
    for form in (L.SCATTER_NODES, L.SCATTER_TILED):
        bs = batched.BatchedStep(MIXED, ns, params, dtype="bf16")
        bs.plan.set_scatter_form(form)
        assert bs.plan.scatter_form() == form
        bs.load(xcs, vps)
        bs.step()
        outs[form] = bs.results()
    for b in range(len(MIXED)):
        for key in ("xcorr", "bc"):
            assert np.array_equal(outs[L.SCATTER_NODES][b][key], outs[L.SCATTER_TILED][b][key]), (b, key)
    # each box's tiled extension equals the single box's
    for b, box in enumerate(MIXED):
        st = stepper.CorrectionStep(box, ns, params, dtype="bf16")
        ref = st.run_numpy(xcs[b], vps[b])
        assert np.array_equal(outs[L.SCATTER_TILED][b]["xcorr"][:3], ref["vcorr"].astype(np.float32)), b
    with pytest.raises(Exception):
        bs.plan.set_scatter_form(L.SCATTER_AUTO)


def test_batched_graph_replay(mods):
    L, batched, _ = mods
    say("batched graph replay")
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=5)
    xcs, vps = batch_inputs(BOXES, seed=10)
    bs = batched.BatchedStep(BOXES, ns, params, dtype="bf16")
    bs.load(xcs, vps)
    b0 = bs.bufs["b"].clone()  # the carried right-hand side the replays start from
    bs.autotune(reps=2)
    bs.step()
    eager = bs.results()
    bs.capture()
    for rep in range(3):
        bs.bufs["b"].copy_(b0)
        bs.bufs["bc"].zero_()
        torch.cuda.synchronize()
        bs.replay()
        got = bs.results()
        for b in range(len(BOXES)):
            assert np.array_equal(got[b]["bc"], eager[b]["bc"]), (rep, b)


def test_fused_gather_forward_single(mods, orc):
    L, _, stepper = mods
    say("fused gather+forward, single box")
    w = syn.cfg2()
    inp = syn.step_inputs(w, seed=3)
    params = syn.mlp_params(165, 256, 81, seed=3)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype="bf16", fused=False)
    ref = st.run_numpy(inp.xc, inp.vprev)
    Y = torch.zeros_like(st.Y)
    L.dnnmg_patch_gather_forward(st.box, st.net, st.xt, st.r, Y)
    torch.cuda.synchronize()
    assert np.array_equal(Y.cpu().numpy().reshape(-1, 81), ref["Y"].astype(np.float32))


def test_cfg3_sized_batch_vs_oracle(mods, orc):
    """The 32-box workload: one box of the batch against the FP64 oracle."""
    L, batched, _ = mods
    boxes = syn.cfg3_boxes(seed=0)
    say(f"cfg3 batch: {len(boxes)} boxes, {sum(b.n_patches for b in boxes)} patches")
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=6)
    xcs, vps = batch_inputs(boxes, seed=20)
    bs = batched.BatchedStep(boxes, ns, params, dtype="bf16")
    bs.load(xcs, vps)
    bs.autotune(reps=2)
    bs.step()
    out = bs.results()
    k = int(np.argmin([b.n_patches for b in boxes]))
    p32 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    vp32 = np.asarray(vps[k], np.float32).astype(np.float64)
    ref = orc.correction_step(boxes[k], ns, p32, xcs[k], vp32)
    e = rel_l2(out[k]["xcorr"][:3] - out[k]["xt"][:3], ref["d"])
    say(f"  box {k} {boxes[k].n}: d rel-L2 vs oracle {e:.2e}")
    assert e <= 2e-2
    assert rel_l2(out[k]["bc"], ref["bc"]) <= 2e-2


LARGE = [syn.BoxSpec(n, (1.0, 1.0, 1.0), 7, 0) for n in [(48, 12, 12), (32, 16, 16), (24, 16, 12), (40, 12, 8),
                                                          (16, 16, 16), (8, 8, 8), (36, 10, 14), (20, 20, 10)]]


def test_batched_large_matches_single(mods):
    """A batch of eight larger uneven boxes (about 300 k fine nodes, several
    workgroups per compute unit in every stage): corrected iterates and
    restricted right-hand sides equal the single-box steps bit for bit."""
    L, batched, stepper = mods
    say("batched large", sum(b.n_fine for b in LARGE), "fine nodes")
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=6)
    xcs, vps = batch_inputs(LARGE, seed=20)
    bs = batched.BatchedStep(LARGE, ns, params, dtype="bf16")
    bs.load(xcs, vps)
    bs.step()
    out = bs.results()
    for b, box in enumerate(LARGE):
        st = stepper.CorrectionStep(box, ns, params, dtype="bf16")
        ref = st.run_numpy(xcs[b], vps[b])
        assert np.array_equal(out[b]["xcorr"][:3], ref["vcorr"].astype(np.float32)), b
        assert np.array_equal(out[b]["xcorr"][3], ref["xt"][3].astype(np.float32)), b
        assert np.array_equal(out[b]["bc"], ref["bc"]), b
