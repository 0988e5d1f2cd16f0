"""GPU training kernels against the oracle: loss gradient, backward pass
(weight and bias gradients), AdamW; BF16 and FP32 networks, ragged sizes."""
import numpy as np
import pytest
import torch

import dnnmg_synth as syn
from gpu_util import dev, f32, rel_l2, say, to_gpu
from test_gpu_parity import pack_net, padded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import paper_2307_14837_amd as L

    assert torch.cuda.is_available()
    return L


def gpu_grads(L, dtype, params, X, T):
    H = params[0].shape[1]
    n = X.shape[0]
    Wp, bias = pack_net(L, dtype, params)
    net = L.make_mlp(dtype, H, Wp, bias)
    xt = torch.float32 if dtype == L.F32 else torch.bfloat16
    Xg = to_gpu(padded(X, 192)).to(xt).contiguous().view(-1)
    Y = torch.empty(n * 81, dtype=torch.float32, device=dev())
    saved = torch.empty(L.saved_bytes(net, n), dtype=torch.uint8, device=dev())
    L.dnnmg_patch_forward(net, n, Xg, 192, Y, saved=saved)
    Tg = to_gpu(f32(T).ravel())
    dY = torch.empty_like(Y)
    L.dnnmg_mse_grad(Y, Tg, dY, n=n)
    dW = [torch.empty(s, dtype=torch.float32, device=dev()) for s in (165 * H, H * H, H * 81)]
    db = [torch.empty(s, dtype=torch.float32, device=dev()) for s in (H, H, 81)]
    ws = torch.empty(L.backward_workspace_bytes(net, n), dtype=torch.uint8, device=dev())
    W2 = to_gpu(f32(params[2]).ravel()); W3 = to_gpu(f32(params[4]).ravel())
    L.dnnmg_patch_backward(net, W2, W3, n, Xg, 192, saved, dY, dW, db, ws)
    out = torch.zeros(1, dtype=torch.float64, device=dev())
    wsn = torch.empty(L.norm2_workspace_bytes(), dtype=torch.uint8, device=dev())
    L.dnnmg_norm2_f64(Y, out, wsn, b=Tg, n=n * 81)
    torch.cuda.synchronize()
    shapes = [(165, H), (H, H), (H, 81)]
    g = []
    for l in range(3):
        g += [dW[l].cpu().numpy().reshape(shapes[l]).astype(np.float64), db[l].cpu().numpy().astype(np.float64)]
    return g, out.item() / n, dY.cpu().numpy().reshape(n, 81)


def oracle_grads(orc, params, X, T):
    p = [f32(q).astype(np.float64) for q in params]
    Y, A1, A2 = orc.mlp_forward(X.astype(np.float64), *p, want_hidden=True)
    loss, dY = orc.mse(Y, T.astype(np.float64))
    dW1, db1, dW2, db2, dW3, db3 = orc.mlp_backward(X.astype(np.float64), p[2], p[4], A1, A2, dY)
    return [dW1, db1, dW2, db2, dW3, db3], loss, dY


@pytest.mark.parametrize("H,n", [(64, 1), (64, 257), (128, 4099), (256, 2048), (512, 700)])
def test_backward_fp32(L, orc, H, n):
    say("backward fp32 H", H, "n", n)
    params = syn.mlp_params(165, H, 81, seed=11, bias_scale=0.1)
    rng = np.random.default_rng(12)
    X = f32(rng.standard_normal((n, 165)))
    T = f32(rng.standard_normal((n, 81)) * 0.5)
    g, loss, dY = gpu_grads(L, L.F32, params, X, T)
    gr, lr_, dYr = oracle_grads(orc, params, X, T)
    assert abs(loss - lr_) <= 1e-5 * abs(lr_)
    assert rel_l2(dY, dYr) <= 1e-5
    for i, (a, b) in enumerate(zip(g, gr)):
        e = rel_l2(a, b)
        say(f"  grad {i} rel-L2 {e:.2e}")
        assert e <= 1e-5, i


@pytest.mark.parametrize("H,n", [(128, 333), (256, 4096), (512, 1500)])
def test_backward_bf16(L, orc, H, n):
    say("backward bf16 H", H, "n", n)
    params = syn.mlp_params(165, H, 81, seed=13, bias_scale=0.1)
    rng = np.random.default_rng(14)
    X = f32(rng.standard_normal((n, 165)))
    T = f32(rng.standard_normal((n, 81)) * 0.5)
    g, loss, _ = gpu_grads(L, L.BF16, params, X, T)
    gr, lr_, _ = oracle_grads(orc, params, X, T)
    assert abs(loss - lr_) <= 2e-2 * abs(lr_)
    for i, (a, b) in enumerate(zip(g, gr)):
        e = rel_l2(a, b)
        say(f"  grad {i} rel-L2 {e:.2e}")
        assert e <= 2e-2, i


def test_backward_deterministic(L):
    say("backward run-to-run identical")
    params = syn.mlp_params(165, 128, 81, seed=3)
    rng = np.random.default_rng(4)
    X = f32(rng.standard_normal((5000, 165))); T = f32(rng.standard_normal((5000, 81)))
    g1, _, _ = gpu_grads(L, L.BF16, params, X, T)
    g2, _, _ = gpu_grads(L, L.BF16, params, X, T)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)


def test_adamw(L, orc):
    say("adamw 10 steps")
    rng = np.random.default_rng(5)
    n = 100003
    th0 = f32(rng.standard_normal(n))
    grads = [f32(rng.standard_normal(n)) for _ in range(10)]
    th = to_gpu(th0.copy()); m = torch.zeros(n, dtype=torch.float32, device=dev()); v = torch.zeros_like(m)
    tr = th0.astype(np.float64); mr = np.zeros(n); vr = np.zeros(n)
    for t, gr in enumerate(grads, start=1):
        L.dnnmg_adamw_step(th, m, v, to_gpu(gr), 1e-3, t, wd=1e-2)
        orc.adamw(tr, mr, vr, gr.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, 1e-2, t)
    torch.cuda.synchronize()
    got = th.cpu().numpy()
    assert np.max(np.abs(got - tr)) <= 1e-6 * np.max(np.abs(tr))


@pytest.mark.parametrize("dtype,H,n,tol", [("fp32", 64, 257, 1e-5), ("bf16", 128, 333, 2e-2)])
def test_autograd_function_matches_oracle(L, orc, dtype, H, n, tol):
    """The network as a torch.autograd.Function over the library's forward and
    backward kernels: gradients of a torch-side MSE loss through
    torch.autograd equal the oracle's chain-rule gradients (pinned by finite
    differences), and the loss matches."""
    from paper_2307_14837_amd import train

    say("autograd function", dtype, "H", H, "n", n)
    params = syn.mlp_params(165, H, 81, seed=21, bias_scale=0.1)
    rng = np.random.default_rng(22)
    X = f32(rng.standard_normal((n, 165)))
    T = f32(rng.standard_normal((n, 81)) * 0.5)
    xt = torch.float32 if dtype == "fp32" else torch.bfloat16
    Xg = to_gpu(padded(X, 192)).to(xt).contiguous()
    ps = [to_gpu(f32(p)).requires_grad_(True) for p in params]
    Y = train.patch_mlp(Xg, *ps, dtype=dtype)
    loss = ((Y - to_gpu(T)) ** 2).sum() / n
    loss.backward()
    torch.cuda.synchronize()
    gr, lr_, _ = oracle_grads(orc, params, X, T)
    assert abs(loss.item() - lr_) <= max(tol, 1e-6) * abs(lr_)
    for i, (p, b) in enumerate(zip(ps, gr)):
        e = rel_l2(p.grad.cpu().numpy().astype(np.float64).reshape(b.shape), b)
        say(f"  grad {i} rel-L2 {e:.2e}")
        assert e <= tol, i


@pytest.mark.parametrize("n", [0, 1, 333, 70001])
def test_mse_grad_with_loss(L, orc, n):
    """The loss gradient and the loss in one pass: dY equals dnnmg_mse_grad's
    bit for bit, the FP64 loss sum equals dnnmg_norm2_f64(Y, T) (same
    partition and order) and the oracle's sum of squares."""
    say("loss gradient with the loss", n)
    rng = np.random.default_rng(9)
    Yh = f32(rng.standard_normal((max(n, 1), 81)))
    Th = f32(rng.standard_normal((max(n, 1), 81)))
    Y, T = to_gpu(Yh.ravel()), to_gpu(Th.ravel())
    dY0 = torch.full_like(Y, float("nan"))
    dY1 = torch.full_like(Y, float("nan"))
    ws = torch.zeros(L.norm2_workspace_bytes(), dtype=torch.uint8, device=dev())
    loss0 = torch.zeros(1, dtype=torch.float64, device=dev())
    loss1 = torch.full((1,), float("nan"), dtype=torch.float64, device=dev())
    L.dnnmg_mse_grad(Y, T, dY0, n=n)
    L.dnnmg_norm2_f64(Y, loss0, ws, b=T, n=n * 81)
    L.dnnmg_mse_grad_loss(Y, T, dY1, loss1, ws, n=n)
    torch.cuda.synchronize()
    m = n * 81
    assert torch.equal(dY0[:m], dY1[:m])
    ref = float(np.sum((Yh[:n].astype(np.float64) - Th[:n].astype(np.float64)) ** 2))
    got, sep = float(loss1.item()), float(loss0.item())
    say(f"  loss {got:.6e} (separate {sep:.6e}, oracle {ref:.6e})")
    assert abs(got - sep) <= 1e-13 * max(abs(sep), 1e-300)
    assert abs(got - ref) <= 1e-12 * max(abs(ref), 1e-300)
