"""Training of the patch network on the GPU with the library's own kernels
(arXiv 2307.14837, Sec. 4.2 "Training of DNN-MG"; AdamW of Sec. 3).

Objective: the mean over patches of ||Y_M - T_M||^2, where the target T_M is
the ground-truth fine velocity minus the prolongated coarse velocity on the
patch's 81 velocity unknowns (the network predicts the correction d).
Each optimisation step runs, on one stream and without host round trips:
forward with saved activations, loss gradient, backward (five products),
AdamW on the FP32 master weights, and re-packing of the low-precision
copies the forward kernels read.  Inputs are standardised per feature
(shift / inv_scale) and the targets by one scalar, folded into the output
layer when the weights are exported.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .stepper import DTYPES, LDX

_XT = {L.F32: torch.float32, L.BF16: torch.bfloat16}


class PatchMLPFunction(torch.autograd.Function):
    """The patch network as a differentiable torch operation whose forward and
    backward run on the library's kernels (dnnmg_patch_forward with saved
    activations; dnnmg_patch_backward, the chain rule through both tanh
    layers of Sec. 3's network).

    apply(X, W1, b1, W2, b2, W3, b3, dtype) -> Y [n][81] FP32.  X [n][192]
    holds the gathered inputs in the network's element type (FP32 or BF16;
    no gradient flows to it); W are the FP32 master weights [fan_in][fan_out]
    and b the FP32 biases.  The forward packs the weights (dnnmg_mlp_prepare)
    and runs the network; the backward takes dL/dY and returns dL/dW and
    dL/db, FP32.  The products of a BF16 network run on BF16 MFMA with FP32
    accumulation (as the library documents); FP8 networks do not train.
    """

    @staticmethod
    def forward(ctx, X, W1, b1, W2, b2, W3, b3, dtype):
        dt = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if dt not in (L.F32, L.BF16):
            raise ValueError("training runs in FP32 or BF16")
        if X.dim() != 2 or X.shape[1] != LDX or X.dtype != _XT[dt]:
            raise ValueError(f"X must be [n][{LDX}] {_XT[dt]}")
        n, H = X.shape[0], W1.shape[1]
        dev = X.device
        Ws = [W1.detach().contiguous(), W2.detach().contiguous(), W3.detach().contiguous()]
        bs = [b1.detach().contiguous(), b2.detach().contiguous(), b3.detach().contiguous()]
        prep = L.mlp_prepare(dt, H, Ws, bs, device=dev)
        Y = torch.empty(n * L.N_OUT, dtype=torch.float32, device=dev)
        saved = torch.empty(max(L.saved_bytes(prep.net, n), 16), dtype=torch.uint8, device=dev)
        X = X.contiguous()
        L.dnnmg_patch_forward(prep.net, n, X, LDX, Y, saved=saved)
        ctx.save_for_backward(X, Ws[1], Ws[2], saved)
        ctx.prep, ctx.n, ctx.H = prep, n, H
        return Y.view(n, L.N_OUT)

    @staticmethod
    def backward(ctx, dY):
        X, W2, W3, saved = ctx.saved_tensors
        n, H, net = ctx.n, ctx.H, ctx.prep.net
        dev = X.device
        f32 = dict(dtype=torch.float32, device=dev)
        dW = [torch.empty(L.N_IN, H, **f32), torch.empty(H, H, **f32), torch.empty(H, L.N_OUT, **f32)]
        db = [torch.empty(H, **f32), torch.empty(H, **f32), torch.empty(L.N_OUT, **f32)]
        ws = torch.empty(max(L.backward_workspace_bytes(net, n), 16), dtype=torch.uint8, device=dev)
        L.dnnmg_patch_backward(net, W2, W3, n, X, LDX, saved, dY.contiguous().view(-1).float(), dW, db, ws)
        return None, dW[0], db[0], dW[1], db[1], dW[2], db[2], None


def patch_mlp(X, W1, b1, W2, b2, W3, b3, dtype="fp32"):
    """Y = N(X) on the library's kernels, differentiable in the parameters."""
    return PatchMLPFunction.apply(X, W1, b1, W2, b2, W3, b3, dtype)


class PatchTrainer:
    def __init__(self, params, dtype="bf16", lr=1e-3, weight_decay=1e-5, betas=(0.9, 0.999), eps=1e-8,
                 device="cuda:0", max_batch=65536):
        self.dev = torch.device(device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        if self.dtype not in (L.F32, L.BF16):
            raise ValueError("training runs in FP32 or BF16")
        self.hidden = int(np.shape(params[0])[1])
        self.lr, self.wd, self.betas, self.eps = lr, weight_decay, betas, eps
        f32 = dict(dtype=torch.float32, device=self.dev)
        # parameters, moments and gradients are views into flat buffers (each
        # tensor padded to 256 bytes; the padding stays zero under AdamW), so
        # one AdamW launch updates them all
        sizes = [int(np.prod(np.shape(p))) for p in params]
        offs, total = [], 0
        for n in sizes:
            offs.append(total)
            total += (n + 63) // 64 * 64
        self._flat = {k: torch.zeros(total, **f32) for k in ("theta", "m", "v", "grad")}
        views = lambda k: [self._flat[k][o:o + n] for o, n in zip(offs, sizes)]
        self.theta, self.m, self.v, self.grad = views("theta"), views("m"), views("v"), views("grad")
        for t, p in zip(self.theta, params):
            t.copy_(torch.as_tensor(np.asarray(p, np.float32)).reshape(-1))
        self.t = 0
        H = self.hidden
        self.Wp = [torch.zeros(L.packed_bytes(self.dtype, H, l), dtype=torch.uint8, device=self.dev) for l in range(3)]
        self.net = L.make_mlp(self.dtype, H, self.Wp, [self.theta[1], self.theta[3], self.theta[5]])
        self._repack()
        self.max_batch = max_batch
        self.Y = torch.zeros(max_batch * L.N_OUT, **f32)
        self.dY = torch.zeros(max_batch * L.N_OUT, **f32)
        self.saved = torch.zeros(L.saved_bytes(self.net, max_batch), dtype=torch.uint8, device=self.dev)
        self.ws = torch.zeros(L.backward_workspace_bytes(self.net, max_batch), dtype=torch.uint8, device=self.dev)
        self.ws_norm = torch.zeros(L.norm2_workspace_bytes(), dtype=torch.uint8, device=self.dev)
        self.loss_dev = torch.zeros(1, dtype=torch.float64, device=self.dev)

    def _repack(self, stream=None):
        for l in range(3):
            L.dnnmg_mlp_pack(self.dtype, self.hidden, l, self.theta[2 * l], self.Wp[l], stream=stream)

    def step(self, X, T, n, stream=None):
        """One AdamW step on a batch: X [n][192] (network dtype), T FP32 [n][81]."""
        if n > self.max_batch:
            raise ValueError("batch larger than max_batch")
        L.dnnmg_patch_forward(self.net, n, X, LDX, self.Y, saved=self.saved, stream=stream)
        # the loss gradient and the loss (for loss()) in one pass
        L.dnnmg_mse_grad_loss(self.Y, T, self.dY, self.loss_dev, self.ws_norm, n=n, stream=stream)
        L.dnnmg_patch_backward(self.net, self.theta[2], self.theta[4], n, X, LDX, self.saved, self.dY,
                               [self.grad[0], self.grad[2], self.grad[4]],
                               [self.grad[1], self.grad[3], self.grad[5]], self.ws, stream=stream)
        self.t += 1
        f = self._flat
        L.dnnmg_adamw_step(f["theta"], f["m"], f["v"], f["grad"], self.lr, self.t, b1=self.betas[0], b2=self.betas[1],
                           eps=self.eps, wd=self.wd, stream=stream)
        self._repack(stream)

    def loss(self, n):
        """Patch loss of the last step (synchronises)."""
        return float(self.loss_dev.item()) / n

    def params(self, target_scale=1.0):
        """Trained parameters as numpy [W1, b1, W2, b2, W3, b3]; the output
        layer is multiplied by the target scale used in training."""
        H = self.hidden
        shapes = [(L.N_IN, H), (H,), (H, H), (H,), (H, L.N_OUT), (L.N_OUT,)]
        out = [t.detach().cpu().numpy().reshape(s).astype(np.float64) for t, s in zip(self.theta, shapes)]
        out[4] = out[4] * target_scale
        out[5] = out[5] * target_scale
        return out


def gather_inputs(box, ns, xc_list, vprev_list, dtype=L.F32, shift=None, inv_scale=None, device="cuda:0"):
    """Network inputs of many steps of one box through the library's
    prolongation, residual and gather kernels: [steps * N_p][192]."""
    dev = torch.device(device)
    nf, nc, npch = L.box_sizes(box)
    xc = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    vp = torch.zeros(3 * nf, dtype=torch.float32, device=dev)
    xt = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    r = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    ws = torch.zeros(L.residual_workspace_bytes(box), dtype=torch.uint8, device=dev)
    X = torch.zeros(len(xc_list) * npch * LDX, dtype=_XT[dtype], device=dev)
    sh = None if shift is None else torch.as_tensor(np.asarray(shift, np.float32)).to(dev)
    sc = None if inv_scale is None else torch.as_tensor(np.asarray(inv_scale, np.float32)).to(dev)
    for s, (c, v) in enumerate(zip(xc_list, vprev_list)):
        xc.copy_(torch.as_tensor(np.asarray(c, np.float64).ravel()))
        vp.copy_(torch.as_tensor(np.asarray(v, np.float32).ravel()))
        L.dnnmg_prolong(box, xc, xt)
        L.dnnmg_residual(box, ns, xt, vp, r, ws)
        L.dnnmg_patch_gather(box, xt, r, X[s * npch * LDX:(s + 1) * npch * LDX], dtype, LDX, sh, sc)
    return X


def feature_stats(X32, n_rows):
    """Per-feature shift and inverse scale from FP32 inputs [n][192] (host)."""
    A = X32.view(n_rows, LDX)[:, : L.N_IN].double().cpu().numpy()
    mu = A.mean(axis=0)
    sd = A.std(axis=0)
    inv = np.where(sd > 1e-12 * np.maximum(1.0, np.abs(mu)), 1.0 / np.where(sd > 0, sd, 1.0), 1.0)
    return mu.astype(np.float32), inv.astype(np.float32)


def plain_correction_pairs(box, ns, inputs, sweeps=4, device="cuda:0"):
    """Training pairs from the plain fine-level method on one box (the
    learned part is trained on data the plain method generates).  For every
    (x^L, v_prev) of `inputs`: b = Rhs(v_prev); x~ = P x^L and r = b - A(x~);
    the plain correction x_V = `sweeps` pressure-held patch-Vanka sweeps from
    x~ (the fallback's correction, taken unconditionally); the network input
    Q(x~, r) and the target Q(x_V - x~) (velocity part, 81 per patch).
    Every step runs in the library's kernels.  Returns FP32 inputs [rows][192]
    (not standardised), targets [rows][81] and the indicator of the plain
    correction eta_V = ||r(x_V)|| / ||r(x~)|| per input."""
    dev = torch.device(device)
    bx, nsp = L.Box.of(box), L.NS.of(ns)
    nf, nc, npch = L.box_sizes(bx)
    f32 = dict(dtype=torch.float32, device=dev)
    xc = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    vp = torch.zeros(3 * nf, **f32)
    xt, r, b, xv, rv = (torch.zeros(4 * nf, **f32) for _ in range(5))
    ws_fb = torch.zeros(L.fallback_workspace_bytes(bx), dtype=torch.uint8, device=dev)
    ws_res = torch.zeros(L.residual_workspace_bytes(bx), dtype=torch.uint8, device=dev)
    ws_n = torch.zeros(2 * L.norm2_workspace_bytes(), dtype=torch.uint8, device=dev)
    norms = torch.ones(2, dtype=torch.float64, device=dev)
    Tpad = torch.zeros(npch * LDX, **f32)
    X = torch.zeros(len(inputs) * npch, LDX, **f32)
    T = torch.zeros(len(inputs) * npch, L.N_OUT, **f32)
    etas = []
    for s, (c, v) in enumerate(inputs):
        xc.copy_(torch.as_tensor(np.asarray(c, np.float64).ravel()))
        vp.copy_(torch.as_tensor(np.asarray(v, np.float32).ravel()))
        L.dnnmg_rhs(bx, nsp, vp, b)
        L.dnnmg_prolong_residual_b(bx, nsp, xc, b, xt, r)
        L.dnnmg_patch_gather(bx, xt, r, X[s * npch:(s + 1) * npch], L.F32, LDX)
        norms.fill_(1.0)  # eta = 1 > theta = 0: the plain correction is taken
        L.dnnmg_fallback_b(bx, nsp, xt, b, norms, xv, ws_fb, theta=0.0, sweeps=sweeps)
        L.dnnmg_residual_b(bx, nsp, xv, b, rv, ws_res)
        L.dnnmg_norm2_pair_f64(r, rv, norms, ws_n)
        dv = xv - xt
        L.dnnmg_patch_gather(bx, dv, dv, Tpad, L.F32, LDX)
        T[s * npch:(s + 1) * npch] = Tpad.view(npch, LDX)[:, :L.N_OUT]
        n = norms.cpu().numpy()
        etas.append(float(np.sqrt(n[1] / n[0])) if n[0] > 0 else 0.0)
    return X, T, etas


def standardisation(X32, n_in=L.N_IN):
    """Per-feature shift and inverse scale (R9 standardisation) of FP32
    inputs [rows][ld]: mean and 1/std over the rows of the first n_in
    columns (constant features keep scale 1)."""
    A = X32[:, :n_in].double()
    mu, sd = A.mean(0), A.std(0)
    ok = sd > 1e-12 * torch.clamp(mu.abs(), min=1.0)
    inv = torch.where(ok, 1.0 / torch.where(ok, sd, torch.ones_like(sd)), torch.ones_like(sd))
    return mu.float(), inv.float()


def distill(box, ns, inputs, hidden, steps=600, batch=65536, lr=1e-3, seed=0, sweeps=4, device="cuda:0"):
    """Trains the patch network on the plain fine-level correction of `box`
    (plain_correction_pairs on `inputs`), BF16 compute with FP32 master
    weights and AdamW, batches of `batch` rows drawn uniformly.  Inputs are
    standardised per feature and the targets by one scalar, folded into the
    output layer of the returned parameters.  Returns (params [W1, b1, W2,
    b2, W3, b3] numpy, shift, inv_scale (numpy FP32 [165]), info)."""
    dev = torch.device(device)
    X, T, etas = plain_correction_pairs(box, ns, inputs, sweeps=sweeps, device=device)
    shift, inv = standardisation(X)
    rows = X.shape[0]
    Z = torch.zeros(rows, LDX, dtype=torch.bfloat16, device=dev)
    Z[:, :L.N_IN] = ((X[:, :L.N_IN] - shift) * inv).to(torch.bfloat16)
    del X
    t_scale = float(T.double().std().item())
    Tn = T / t_scale
    params = [np.asarray(p) for p in _init_params(hidden, seed)]
    tr = PatchTrainer(params, dtype="bf16", lr=lr, weight_decay=1e-5, max_batch=batch, device=device)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    bsz = min(batch, rows)
    for _ in range(steps):
        idx = torch.randint(0, rows, (bsz,), device=dev, generator=g)
        tr.step(Z[idx].contiguous().view(-1), Tn[idx].contiguous().view(-1), bsz)
    info = {"rows": rows, "steps": steps, "batch": bsz, "final_loss": tr.loss(bsz), "target_scale": t_scale,
            "plain_correction_eta": etas}
    return tr.params(target_scale=t_scale), shift.cpu().numpy(), inv.cpu().numpy(), info


def _init_params(hidden, seed):
    """N(0, 1/fan_in) weights, zero biases, the output layer scaled by 0.1
    (a small initial correction)."""
    rng = np.random.default_rng(seed)
    out = []
    for fi, fo in ((L.N_IN, hidden), (hidden, hidden), (hidden, L.N_OUT)):
        out += [rng.standard_normal((fi, fo)) / np.sqrt(fi), np.zeros(fo)]
    out[4] *= 0.1
    return out


def _doubled(box):
    """The box with twice the cells per axis: its coarse mesh is the fine
    mesh of `box`, so the coarse-step solver solves on that mesh."""
    b = L.Box.of(box)
    out = L.Box()
    for a in range(3):
        out.n[a] = 2 * b.n[a]
        out.len[a] = b.len[a]
    out.periodic_mask, out.dirichlet_mask = b.periodic_mask, b.dirichlet_mask
    return out


def teacher_forced(box, ns, v0, xc0, steps, fine_bc, coarse_bc, opts=None, device="cuda:0", log=None):
    """Teacher-forced data of the plain method on the GPU (the reading of
    Sec. 4.2 that the oracle's CPU solver follows):
      F_n   = Rhs_fine(vbar_{n-1})
      x^L_n : A_coarse(x^L_n) = R F_n   (Dirichlet velocity rows zero)
      xbar_n: A_fine(xbar_n) = F_n      (ground truth)
    Both solves are dnnmg_coarse_solve (the fine one on the box with twice
    the cells, whose coarse mesh is this box's fine mesh), each started from
    the previous step's solution with the Dirichlet data (fine_bc /
    coarse_bc: (mask [4][N] bool, values [4][N]) on the fine / coarse nodes).
    Returns xc (list of FP64 [4][n_coarse] GPU tensors, steps 1..n), vbar
    (list of FP32 [3][n_fine], vbar[0] = v0), pbar (FP32 [n_fine], steps
    1..n) and the residual norms of each solve."""
    dev = torch.device(device)
    bx, nsp = L.Box.of(box), L.NS.of(ns)
    fbx = _doubled(bx)
    nf, nc, _ = L.box_sizes(bx)
    opts = opts or L.coarse_opts(newton_its=10)
    ws_c = torch.empty(L.coarse_workspace_bytes(bx, opts), dtype=torch.uint8, device=dev)
    ws_f = torch.empty(L.coarse_workspace_bytes(fbx, opts), dtype=torch.uint8, device=dev)
    fm = torch.as_tensor(np.asarray(fine_bc[0], bool).reshape(-1), device=dev)
    fv = torch.as_tensor(np.asarray(fine_bc[1], np.float64).reshape(-1), device=dev)
    cm = torch.as_tensor(np.asarray(coarse_bc[0], bool).reshape(-1), device=dev)
    cv = torch.as_tensor(np.asarray(coarse_bc[1], np.float64).reshape(-1), device=dev)
    F = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    bL = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    xc = torch.as_tensor(np.asarray(xc0, np.float64).reshape(-1)).to(dev)
    xf = torch.zeros(4 * nf, dtype=torch.float64, device=dev)
    xf[:3 * nf] = torch.as_tensor(np.asarray(v0, np.float64).reshape(-1)).to(dev)
    vbar = [xf[:3 * nf].float().view(3, nf).clone()]
    xcs, pbar, norms = [], [], []
    res_c = torch.zeros(opts.newton_its + 1, dtype=torch.float64, device=dev)
    res_f = torch.zeros_like(res_c)
    for n in range(1, steps + 1):
        L.dnnmg_rhs(bx, nsp, vbar[-1].reshape(-1).contiguous(), F)
        L.dnnmg_restrict(bx, F, bL)
        bL.masked_fill_(cm & (torch.arange(4 * nc, device=dev) < 3 * nc), 0.0)
        xc = torch.where(cm, cv, xc)
        L.dnnmg_coarse_solve(bx, nsp, bL, xc, opts, ws_c, res_c)
        bF = F.double()
        bF.masked_fill_(fm & (torch.arange(4 * nf, device=dev) < 3 * nf), 0.0)
        xf = torch.where(fm, fv, xf)
        L.dnnmg_coarse_solve(fbx, nsp, bF, xf, opts, ws_f, res_f)
        xcs.append(xc.clone())
        vbar.append(xf[:3 * nf].float().view(3, nf).clone())
        pbar.append(xf[3 * nf:].float().clone())
        norms.append((res_c.cpu().numpy(), res_f.cpu().numpy()))
        if log and (n == 1 or n % 25 == 0 or n == steps):
            log(f"teacher-forced step {n}/{steps}: coarse |r| {norms[-1][0][0]:.2e} -> {norms[-1][0][-1]:.2e}, "
                f"fine |r| {norms[-1][1][0]:.2e} -> {norms[-1][1][-1]:.2e}")
    return xcs, vbar, pbar, norms


def gather_targets(box, xc_list, vnext_list, device="cuda:0"):
    """Training targets of many steps: Q(vbar_n - P x^L_n) on each patch (the
    81 velocity unknowns; Sec. 4.2 training objective), FP32 [steps * N_p][81]."""
    dev = torch.device(device)
    nf, nc, npch = L.box_sizes(box)
    xt = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    dv = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    Tpad = torch.zeros(npch * LDX, dtype=torch.float32, device=dev)
    T = torch.zeros(len(xc_list) * npch, L.N_OUT, dtype=torch.float32, device=dev)
    for s, (c, v) in enumerate(zip(xc_list, vnext_list)):
        L.dnnmg_prolong(box, torch.as_tensor(c).to(dev, torch.float64).contiguous().view(-1), xt)
        dv[:3 * nf] = torch.as_tensor(v).to(dev, torch.float32).reshape(-1) - xt[:3 * nf]
        L.dnnmg_patch_gather(box, dv, dv, Tpad, L.F32, LDX)
        T[s * npch:(s + 1) * npch] = Tpad.view(npch, LDX)[:, :L.N_OUT]
    return T


def paper_inputs(box, ns, xc_list, vprev_list, hidden=512, device="cuda:0"):
    """The paper's network inputs of many steps (Sec. 4.2: velocities,
    pressure, the four residuals and 24 geometry features per patch) through
    the library's prolongation, residual and dnnmg_patch_gather_paper, not
    standardised: FP32 [steps * N_p][ldx]."""
    dev = torch.device(device)
    nf, nc, npch = L.box_sizes(box)
    ldx = L.deepnet_widths(240, hidden, L.N_OUT)[0]
    xc = torch.zeros(4 * nc, dtype=torch.float64, device=dev)
    vp = torch.zeros(3 * nf, dtype=torch.float32, device=dev)
    xt = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    r = torch.zeros(4 * nf, dtype=torch.float32, device=dev)
    ws = torch.zeros(L.residual_workspace_bytes(box), dtype=torch.uint8, device=dev)
    X = torch.zeros(len(xc_list) * npch, ldx, dtype=torch.float32, device=dev)
    for s, (c, v) in enumerate(zip(xc_list, vprev_list)):
        xc.copy_(torch.as_tensor(c).to(dev, torch.float64).reshape(-1))
        vp.copy_(torch.as_tensor(v).to(dev, torch.float32).reshape(-1))
        L.dnnmg_prolong(box, xc, xt)
        L.dnnmg_residual(box, ns, xt, vp, r, ws)
        L.dnnmg_patch_gather_paper(box, 1, xt, r, X[s * npch:(s + 1) * npch], L.F32, ldx)
    return X


class PaperNet(torch.nn.Module):
    """The paper's network form for training (Sec. 3): no biases, batch
    normalisation before each tanh (batch statistics in training), skip
    connections on the hidden layers after the first."""

    def __init__(self, n_in, hidden, n_out, depth=8):
        super().__init__()
        self.lin = torch.nn.ModuleList([torch.nn.Linear(n_in, hidden, bias=False)] +
                                       [torch.nn.Linear(hidden, hidden, bias=False) for _ in range(depth - 1)])
        self.bn = torch.nn.ModuleList([torch.nn.BatchNorm1d(hidden, eps=1e-5) for _ in range(depth)])
        self.out = torch.nn.Linear(hidden, n_out, bias=False)

    def forward(self, x):
        a = x
        for i, (lin, bn) in enumerate(zip(self.lin, self.bn)):
            h = torch.tanh(bn(lin(a)))
            a = h if i == 0 else h + a
        return self.out(a)


def train_paper_network(X, T, n_in=240, hidden=512, depth=8, steps=400, batch=65536, lr=1e-3, seed=0,
                        device="cuda:0"):
    """Trains the paper's network form with torch autograd (FP32, AdamW) on
    standardised inputs X [rows][>= n_in] and targets T [rows][81] (scaled
    by one scalar, folded back into the output layer).  The batch
    normalisations' statistics are then taken over all rows (their running
    averages at the final weights), for the folded inference of
    dnnmg_deepnet_prepare.  Returns ((Ws, gammas, betas, means, stds),
    module, target scale, final loss)."""
    dev = torch.device(device)
    torch.manual_seed(seed)
    net = PaperNet(n_in, hidden, L.N_OUT, depth).to(dev)
    t_scale = float(T.double().std().item())
    Tn = T / t_scale
    Xi = X[:, :n_in].contiguous()
    opt = torch.optim.AdamW(net.parameters(), lr=lr, weight_decay=1e-5)
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    rows = Xi.shape[0]
    bsz = min(batch, rows)
    loss = None
    for _ in range(steps):
        idx = torch.randint(0, rows, (bsz,), device=dev, generator=g)
        opt.zero_grad(set_to_none=True)
        loss = torch.mean(torch.sum((net(Xi[idx]) - Tn[idx]) ** 2, dim=1))
        loss.backward()
        opt.step()
    # population statistics of every normalisation at the final weights
    for bn in net.bn:
        bn.reset_running_stats()
        bn.momentum = None
    with torch.no_grad():
        for b0 in range(0, rows, bsz):
            net(Xi[b0:b0 + bsz])
    net.eval()
    Ws = [lin.weight.detach().t().double().cpu().numpy() for lin in net.lin]
    Ws.append(net.out.weight.detach().t().double().cpu().numpy() * t_scale)
    gammas = [bn.weight.detach().double().cpu().numpy() for bn in net.bn]
    betas = [bn.bias.detach().double().cpu().numpy() for bn in net.bn]
    means = [bn.running_mean.detach().double().cpu().numpy() for bn in net.bn]
    stds = [np.sqrt(bn.running_var.detach().double().cpu().numpy() + bn.eps) for bn in net.bn]
    return (Ws, gammas, betas, means, stds), net, t_scale, float(loss.item())
