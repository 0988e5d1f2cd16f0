"""Boundary calls added for setup and capture: dnnmg_mlp_prepare (packing and
the FP8 per-tensor scales chosen in the library) and the HIP-graph capture
entry points, through the C ABI."""
import ctypes

import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, f32, say, to_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    return L


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8"])
def test_mlp_prepare_scales_and_packing(L, dtype):
    """The FP8 weight scale is max |W2| / 448 of the FP32 weights, exactly as
    FP32 arithmetic gives it; the tanh-output scale is 1/448; the packed
    layers equal dnnmg_mlp_pack's with those scales, bit for bit."""
    from paper_2307_14837_amd.stepper import DTYPES

    H = 256
    dt = DTYPES[dtype]
    params = syn.mlp_params(165, H, 81, seed=3, bias_scale=0.1)
    W32 = [to_gpu(f32(params[2 * l])) for l in range(3)]
    bias = [to_gpu(f32(params[2 * l + 1])) for l in range(3)]
    prep = L.mlp_prepare(dt, H, W32, bias)
    net = prep.net
    amax = np.float32(np.abs(f32(params[2])).max())
    want = np.float32(amax / np.float32(448.0)) if dtype == "fp8" else np.float32(1.0)
    say(f"{dtype}: w_scale {list(net.w_scale)} a_scale {list(net.a_scale)}")
    assert np.float32(net.w_scale[1]) == want
    assert np.float32(net.a_scale[1]) == (np.float32(1.0 / 448.0) if dtype == "fp8" else 1.0)
    assert net.n_in == 165 and net.n_out == 81 and net.hidden == H and net.dtype == dt
    for l in range(3):
        ref = torch.zeros_like(prep.Wp[l])
        L.dnnmg_mlp_pack(dt, H, l, W32[l], ref, w_scale=float(net.w_scale[l]))
        torch.cuda.synchronize()
        assert torch.equal(ref, prep.Wp[l]), l
        assert net.W[l] == prep.Wp[l].data_ptr() and net.b[l] == bias[l].data_ptr()


def test_mlp_prepare_rejects_nonfinite_fp8_weights(L):
    H = 128
    params = syn.mlp_params(165, H, 81, seed=1)
    params[2] = params[2].copy()
    params[2][3, 5] = np.nan
    W32 = [to_gpu(f32(params[2 * l])) for l in range(3)]
    bias = [to_gpu(f32(params[2 * l + 1])) for l in range(3)]
    with pytest.raises(L.DnnmgError) as ei:
        L.mlp_prepare(L.FP8_E4M3, H, W32, bias)
    assert "W2" in str(ei.value)


def test_graph_capture_replay_c_abi(L):
    """A right-hand side and a restriction recorded with
    dnnmg_graph_capture_begin/_end and replayed three times, with eager work
    and synchronisation between the replays: every replay equals the eager
    result, and reads the buffers' current contents."""
    box = syn.channel_box((8, 4, 4))
    ns = syn.NSParams(1e-3, 0.005)
    nf, nc = box.n_fine, box.n_coarse
    rng = np.random.default_rng(5)
    v = to_gpu(f32(rng.standard_normal(3 * nf)))
    b = torch.zeros(4 * nf, dtype=torch.float32, device=dev())
    bc = torch.zeros(4 * nc, dtype=torch.float64, device=dev())

    def work():
        L.dnnmg_rhs(box, ns, v, b)
        L.dnnmg_restrict(box, b, bc)

    work()
    torch.cuda.synchronize()
    eager = (b.clone(), bc.clone())
    g = L.capture_graph(work)
    for rep in range(3):
        b.fill_(float("nan"))
        bc.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b, eager[0]) and torch.equal(bc, eager[1]), rep
    # a changed input is read by the next replay
    v.mul_(2.0)
    work()
    torch.cuda.synchronize()
    eager2 = bc.clone()
    bc.zero_()
    g.replay()
    torch.cuda.synchronize()
    assert torch.equal(bc, eager2)
    # capture on the legacy default stream is refused before anything runs
    lib = L._lib.lib()
    assert lib.dnnmg_graph_capture_begin(None) == -1
    h = ctypes.c_void_p()
    assert lib.dnnmg_graph_capture_end(None, ctypes.byref(h)) == -1
