"""Allocation-free residual against b (dnnmg_residual_b_noalloc) against the
workspace form dnnmg_residual_b, through the C ABI: bit-for-bit equal on two
calls in a row (the second on a smaller box, so the built-in scratch holds
the first call's corner sums and tile flags), and within the parity bar of
the FP64 oracle.  Collected last: it shares the library's per-GPU scratch.
"""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, f32, rel_l2, say, to_gpu

pytestmark = pytest.mark.gpu


def _case(L, orc, box, seed):
    ns = syn.NSParams(0.05, 0.02, 0.5, 0.8)
    rng = np.random.default_rng(seed)
    # a general iterate (not prolongated), so every cell has LPS terms and the
    # corner sums in the scratch are written and read
    x = f32(rng.standard_normal((4, box.n_fine)))
    vp = f32(x[:3] + 0.3 * rng.standard_normal((3, box.n_fine)))
    nf = box.n_fine
    xg, vpg = to_gpu(x.ravel()), to_gpu(vp.ravel())
    b = torch.empty(4 * nf, dtype=torch.float32, device=dev())
    L.dnnmg_rhs(box, ns, vpg, b)
    ws = torch.empty(L.residual_workspace_bytes(box), dtype=torch.uint8, device=dev())
    r_ws = torch.full((4 * nf,), float("nan"), dtype=torch.float32, device=dev())
    r_na = torch.full((4 * nf,), float("nan"), dtype=torch.float32, device=dev())
    L.dnnmg_residual_b(box, ns, xg, b, r_ws, ws)
    L.dnnmg_residual_b_noalloc(box, ns, xg, b, r_na)
    torch.cuda.synchronize()
    a, c = r_na.cpu().numpy(), r_ws.cpu().numpy()
    assert np.array_equal(a.view(np.uint32), c.view(np.uint32)), "no-alloc form differs from the workspace form"
    ref = orc.residual(box, ns, x.astype(np.float64), vp.astype(np.float64))
    e = rel_l2(a.reshape(4, -1), ref)
    say(f"  {box.n} rel-L2 vs oracle {e:.2e}")
    assert e <= 1e-5


def test_noalloc_residual_b_two_calls(orc):
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    big = syn.channel_box((24, 8, 6))
    small = syn.BoxSpec((6, 4, 2), (1.0, 0.7, 0.4), 7, 0)
    assert small.n_patches < big.n_patches
    say("no-alloc residual_b: large box, then a smaller one")
    _case(L, orc, big, 11)
    _case(L, orc, small, 12)


def test_noalloc_rejects_oversized_box():
    import paper_2307_14837_amd as L

    # 128 x 64 x 64 coarse cells need about 64 MiB of corner sums: rejected on
    # the host before anything is enqueued (no device pointer is touched)
    box = syn.channel_box((128, 64, 64))
    assert L.residual_workspace_bytes(box) > L.NOALLOC_SCRATCH_BYTES
    x = torch.zeros(4 * box.n_fine, dtype=torch.float32, device=dev())
    with pytest.raises(L.DnnmgError) as ei:
        L.dnnmg_residual_b_noalloc(box, syn.NSParams(1e-3, 0.01), x, x.clone(), x.clone())
    assert "scratch" in str(ei.value)
