"""One DNN-MG correction step on the GPU (arXiv 2307.14837, Algorithm 1 after
the coarse solve): prolongate -> fine residual -> gather Q -> patch network ->
extension L (plus v~) -> right-hand side -> restriction, optionally followed
by the residual indicator (residual of the corrected state and two FP64
norms).  Every arithmetic step runs in libdnnmg's HIP kernels; this module
only owns device buffers (torch allocations), packs the network once and can
capture the whole step in a HIP graph.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L

DTYPES = {"fp32": L.F32, "bf16": L.BF16, "fp8": L.FP8_E4M3}
_TORCH = {L.F32: torch.float32, L.BF16: torch.bfloat16, L.FP8_E4M3: torch.uint8}
LDX = L.IN_PAD  # 192: K padded for the MFMA granule


class CorrectionStep:
    """Buffers and launch sequence of one correction step for one box.

    params: [W1, b1, W2, b2, W3, b3] (numpy or torch, W as [fan_in][fan_out]).
    shift / inv_scale: per-feature standardisation of the 165 inputs (None =
    identity).  carry_rhs (default): the step's residuals are r = b - A(x)
    with b the right-hand side the previous step computed (load() computes
    the first one from vprev), so the terms of the previous velocity are
    evaluated once per step, not again in every residual; carry_rhs=False
    builds them from vprev in each residual instead.  The network is packed by
    the library (dnnmg_mlp_prepare), which also picks the FP8 scales.
    """

    def __init__(self, box, ns, params, dtype="bf16", device="cuda:0", shift=None, inv_scale=None,
                 indicator=False, theta=1.0, fallback_sweeps=4, fused=True, carry_rhs=None, levels=1,
                 network="mlp"):
        self.box = L.Box.of(box)
        self.ns = L.NS.of(ns)
        self.dev = torch.device(device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        # levels = J: the prediction J levels above the coarse mesh (Sec. 4.2);
        # fbox is the box whose own fine mesh is level L + J (the residual,
        # Rhs and fallback run on it)
        self.levels = int(levels)
        self.fbox = L.level_box(self.box, self.levels)
        self.nf, self.nc, self.np = L.level_sizes(self.box, self.levels)
        # network "mlp": the 3-layer tanh network of the configurations;
        # "paper": the paper's form (Sec. 3: batch normalisation, skip
        # connections, D hidden layers) on its inputs (Sec. 4.2), params =
        # (Ws, gammas, betas, means, stds)
        self.network = network
        if network == "paper":
            Ws = params[0]
            self.n_in, self.n_out = int(np.shape(Ws[0])[0]), int(np.shape(Ws[-1])[1])
            self.ldx = L.deepnet_widths(self.n_in, int(np.shape(Ws[0])[1]), self.n_out)[0]
            self.hidden = int(np.shape(Ws[0])[1])
        else:
            self.n_in, self.n_out, self.ldx = L.LEVEL_IO[self.levels]
            self.hidden = int(np.shape(params[0])[1])
        self.indicator = indicator
        # fused: the gather runs inside the network kernel (no X round trip;
        # built for one-level patches)
        self.fused = bool(fused) and self.levels == 1 and network == "mlp"
        self.carry_rhs = True if carry_rhs is None else bool(carry_rhs)
        f32 = dict(dtype=torch.float32, device=self.dev)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.xc = torch.zeros(4 * self.nc, **f64)
        self.xt = torch.zeros(4 * self.nf, **f32)       # prolongated (u, v, w, p)
        self.vprev = torch.zeros(3 * self.nf, **f32)
        self.r = torch.zeros(4 * self.nf, **f32)
        self.ws_res = torch.zeros(L.residual_workspace_bytes(self.fbox), dtype=torch.uint8, device=self.dev)
        # level L + 1 of the fused two-level prolongation and residual
        nws = L.prolong_residual_b_levels_workspace_bytes(self.box, self.levels)
        self.ws_pr = torch.zeros(nws, dtype=torch.uint8, device=self.dev) if nws else None
        # FP8 networks take BF16 inputs (their first layer is BF16)
        self.xdtype = L.F32 if self.dtype == L.F32 else L.BF16
        self.X = torch.zeros(self.np * self.ldx, dtype=_TORCH[self.xdtype], device=self.dev)
        self.Y = torch.zeros(self.np * self.n_out, **f32)
        self.xcorr = torch.zeros(4 * self.nf, **f32)    # (v~ + d, p~)
        self.b = torch.zeros(4 * self.nf, **f32)
        self.bc = torch.zeros(4 * self.nc, **f64)
        self.theta, self.fallback_sweeps = float(theta), int(fallback_sweeps)
        if indicator:
            self.r2 = torch.zeros(4 * self.nf, **f32)
            self.norms = torch.zeros(2, **f64)
            self.ws_norm = torch.zeros(2 * L.norm2_workspace_bytes(), dtype=torch.uint8, device=self.dev)
            self.ws_fb = torch.zeros(L.fallback_workspace_bytes(self.fbox), dtype=torch.uint8, device=self.dev)
            self.fell_back = torch.zeros(1, dtype=torch.int32, device=self.dev)
            # the step's right-hand side, kept for the fallback while b takes
            # the next one (carried form)
            self.b_prev = torch.zeros(4 * self.nf, **f32) if self.carry_rhs else None
        self.shift = None if shift is None else torch.as_tensor(np.asarray(shift, np.float32)).to(self.dev)
        self.inv_scale = None if inv_scale is None else torch.as_tensor(np.asarray(inv_scale, np.float32)).to(self.dev)
        self.set_params(params)
        self.graph = None

    # ------------------------------------------------------------- network --
    def set_params(self, params):
        H = self.hidden
        if self.network == "paper":
            # batch normalisations folded into the packed layers by the library
            self.deep = L.DeepNet(self.dtype, *params, device=self.dev)
            return
        W32 = [torch.as_tensor(np.asarray(params[2 * l], np.float32)).contiguous().to(self.dev) for l in range(3)]
        bias = [torch.as_tensor(np.asarray(params[2 * l + 1], np.float32)).contiguous().to(self.dev) for l in range(3)]
        # packing and the per-tensor scales of the precision scheme are the
        # library's (dnnmg_mlp_prepare)
        self.prepared = L.mlp_prepare(self.dtype, H, W32, bias, device=self.dev, n_in=self.n_in, n_out=self.n_out)
        self.W32, self.bias, self.Wp = self.prepared.W32, self.prepared.bias, self.prepared.Wp
        self.net = self.prepared.net
        self.w_scale = [float(self.net.w_scale[l]) for l in range(3)]

    # ---------------------------------------------------------------- step --
    def load(self, xc, vprev):
        self.xc.copy_(torch.as_tensor(np.asarray(xc, np.float64).ravel()))
        self.vprev.copy_(torch.as_tensor(np.asarray(vprev, np.float32).ravel()))
        if self.carry_rhs:
            # the right-hand side of the previous velocity, as the previous
            # step would have left it
            L.dnnmg_rhs(self.fbox, self.ns, self.vprev, self.b)

    def step(self, stream=None):
        if self.levels != 1 or self.network != "mlp":
            return self._step_levels(stream)
        box, ns = self.box, self.ns
        # x~ = P xc and r = F - A(x~) in one pass (no LPS terms on a prolongation)
        if self.carry_rhs:
            L.dnnmg_prolong_residual_b(box, ns, self.xc, self.b, self.xt, self.r, stream=stream)
        else:
            L.dnnmg_prolong_residual(box, ns, self.xc, self.vprev, self.xt, self.r, stream=stream)
        if self.fused:
            L.dnnmg_patch_gather_forward(box, self.net, self.xt, self.r, self.Y, self.shift, self.inv_scale,
                                         stream=stream)
        else:
            L.dnnmg_patch_gather(box, self.xt, self.r, self.X, self.xdtype, LDX, self.shift, self.inv_scale,
                                 stream=stream)
            L.dnnmg_patch_forward(self.net, self.np, self.X, LDX, self.Y, stream=stream)
        # corrected iterate (v~ + d, p~)
        L.dnnmg_scatter_avg(box, self.Y, self.xcorr, vbase=self.xt, stream=stream)
        self._indicator_rhs(box, stream)
        L.dnnmg_restrict(box, self.b, self.bc, stream=stream)

    def _indicator_rhs(self, fb, stream):
        """[Indicator and fallback,] then b = Rhs(v_corr) on the fine box fb.
        eta = ||r(x_corr)|| / ||r(x~)||; above theta the plain fine correction
        replaces the network's (decided on the device).  Carried form: the
        indicator's residual and the next Rhs are one pass (b replaced in
        place, its old value kept in b_prev for the fallback), and the Rhs is
        taken again only where the fallback changed x_corr."""
        ns = self.ns
        if not self.indicator:
            L.dnnmg_rhs(fb, ns, self.xcorr, self.b, stream=stream)
            return
        if self.carry_rhs:
            L.dnnmg_residual_rhs_b(fb, ns, self.xcorr, self.b, self.r2, self.ws_res, b_save=self.b_prev,
                                   stream=stream)
            L.dnnmg_norm2_pair_f64(self.r, self.r2, self.norms, self.ws_norm, stream=stream)
            L.dnnmg_fallback_b(fb, ns, self.xt, self.b_prev, self.norms, self.xcorr, self.ws_fb, theta=self.theta,
                               sweeps=self.fallback_sweeps, flag_out=self.fell_back, stream=stream)
            L.dnnmg_rhs_if(fb, ns, self.xcorr, self.b, self.fell_back, stream=stream)
            return
        L.dnnmg_residual(fb, ns, self.xcorr, self.vprev, self.r2, self.ws_res, stream=stream)
        L.dnnmg_norm2_pair_f64(self.r, self.r2, self.norms, self.ws_norm, stream=stream)
        L.dnnmg_fallback(fb, ns, self.xt, self.vprev, self.norms, self.xcorr, self.ws_fb, theta=self.theta,
                         sweeps=self.fallback_sweeps, flag_out=self.fell_back, stream=stream)
        L.dnnmg_rhs(fb, ns, self.xcorr, self.b, stream=stream)

    def _step_levels(self, stream=None):
        """The step with the prediction J levels above the coarse mesh (and
        the step with the paper's network at any J): x~ = P^J x^L, the
        residual of level L + J (on fbox, against the carried right-hand
        side or from v_prev), Q and the network on the J-level patches, L
        back to level L + J, [indicator], Rhs on fbox, b^L = (P^J)^T b."""
        box, fb, ns, J = self.box, self.fbox, self.ns, self.levels
        if self.carry_rhs:
            # prolongation and residual in one pass (J = 2: level L + 1
            # first), the local projection terms vanishing on x~
            L.dnnmg_prolong_residual_b_levels(box, J, ns, self.xc, self.b, self.xt, self.r, ws=self.ws_pr,
                                              stream=stream)
        else:
            L.dnnmg_prolong_levels(box, J, self.xc, self.xt, stream=stream)
            if self.carry_rhs:
                L.dnnmg_residual_b(fb, ns, self.xt, self.b, self.r, self.ws_res, stream=stream)
            else:
                L.dnnmg_residual(fb, ns, self.xt, self.vprev, self.r, self.ws_res, stream=stream)
        if self.network == "paper":
            L.dnnmg_patch_gather_paper(box, J, self.xt, self.r, self.X, self.xdtype, self.ldx, self.shift,
                                       self.inv_scale, stream=stream)
            L.dnnmg_deepnet_forward(self.deep, self.np, self.X, self.ldx, self.Y, stream=stream)
        else:
            L.dnnmg_patch_gather_levels(box, J, self.xt, self.r, self.X, self.xdtype, self.ldx, self.shift,
                                        self.inv_scale, stream=stream)
            L.dnnmg_patch_forward(self.net, self.np, self.X, self.ldx, self.Y, stream=stream)
        L.dnnmg_scatter_avg_levels(box, J, self.Y, self.xcorr, vbase=self.xt, stream=stream)
        self._indicator_rhs(fb, stream)
        L.dnnmg_restrict_levels(box, J, self.b, self.bc, stream=stream)

    def attach_coarse(self, opts, coarse_bc):
        """Makes time_step() a whole time step of Algorithm 1 on the GPU: the
        coarse problem A(x^L) = b^L (b^L the restriction of the previous
        step's fine Rhs, left in bc, with its Dirichlet velocity rows zero)
        solved by dnnmg_coarse_solve from the previous x^L with the Dirichlet
        data coarse_bc = (mask [4][n_coarse] bool, values [4][n_coarse]),
        then step().  One-level prediction with the carried right-hand side
        only."""
        if self.levels != 1 or not self.carry_rhs:
            raise ValueError("the GPU time step is built for J = 1 with the carried right-hand side")
        mask = torch.as_tensor(np.asarray(coarse_bc[0], bool).reshape(-1), device=self.dev)
        vals = torch.as_tensor(np.asarray(coarse_bc[1], np.float64).reshape(-1), device=self.dev)
        self.c_opts = opts
        self.c_keep = (~mask).double()            # 0 on Dirichlet entries
        self.c_dir = torch.where(mask, vals, torch.zeros_like(vals))
        self.c_keep_rows = self.c_keep.clone()    # b^L: Dirichlet velocity rows zero
        self.bL = torch.zeros_like(self.bc)
        self.c_ws = torch.empty(L.coarse_workspace_bytes(self.box, opts), dtype=torch.uint8, device=self.dev)
        self.c_res = torch.zeros(opts.newton_its + 1, dtype=torch.float64, device=self.dev)
        # the restriction of the loaded Rhs, as the previous step leaves it
        L.dnnmg_restrict(self.box, self.b, self.bc)

    def time_step(self, stream=None):
        """Coarse solve, then the correction step (attach_coarse first).  The
        Dirichlet handling uses in-place elementwise products only, so the
        whole time step can be recorded into one graph."""
        s = torch.cuda.current_stream(self.dev) if stream is None else stream
        with torch.cuda.stream(s):
            self.bL.copy_(self.bc).mul_(self.c_keep_rows)
            self.xc.mul_(self.c_keep).add_(self.c_dir)
        L.dnnmg_coarse_solve(self.box, self.ns, self.bL, self.xc, self.c_opts, self.c_ws, self.c_res, stream=s)
        self.step(s)

    def capture(self, full=False):
        """Record step() (full: time_step()) into a HIP graph through the
        library's capture calls (one eager warm-up run first)."""
        fn = (lambda: self.time_step(torch.cuda.current_stream(self.dev))) if full else self.step
        self.graph = L.capture_graph(fn, device=self.dev)
        return self.graph

    def replay(self, stream=None):
        self.graph.replay(stream)

    def run_numpy(self, xc, vprev):
        self.load(xc, vprev)
        self.step()
        torch.cuda.synchronize(self.dev)
        xt = self.xt.cpu().numpy().reshape(4, -1).astype(np.float64)
        xcorr = self.xcorr.cpu().numpy().reshape(4, -1).astype(np.float64)
        out = {
            "xt": xt,
            "r": self.r.cpu().numpy().reshape(4, -1).astype(np.float64),
            "Y": self.Y.cpu().numpy().reshape(-1, self.n_out).astype(np.float64),
            "vcorr": xcorr[:3],
            "d": xcorr[:3] - xt[:3],
            "b": self.b.cpu().numpy().reshape(4, -1).astype(np.float64),
            "bc": self.bc.cpu().numpy().reshape(4, -1),
            "vprev32": self.vprev.cpu().numpy().reshape(3, -1).astype(np.float64),
        }
        if self.indicator:
            n = self.norms.cpu().numpy()
            out["eta"] = float(np.sqrt(n[1] / n[0])) if n[0] > 0 else float("inf")
            out["fell_back"] = int(self.fell_back.item())
        return out


class Q2CorrectionStep:
    """One correction step of Algorithm 1 on the paper's discretisation
    (Sec. 2.2: Q2/Q2 elements on curved hexahedra, LPS with pi_h: Q2 -> Q1):
    x~ = P xc (Q2 interpolation); r = b - A(x~); X = Q(x~, r, geometry);
    Y = N(X); x_corr = (v~ + L(Y), p~); optionally the indicator's residual
    r(x_corr) and the two FP64 norms; b = Rhs(v_corr); bc = R b.

    The fine Q2 elements are the patches (27 nodes each), so the network,
    the dof map and the extension are those of the Q1 step.  coords: node
    positions [3][n_fine] (FP64).  b is carried from step to step as in the
    Q1 step (load() computes the first one from vprev).  The fallback of the
    Q1 step (its patch-Vanka sweeps are built for Q1) is not part of this
    step: with indicator=True, eta is computed and reported only.
    network "mlp": the 165-H-H-81 network (geometry inputs: mean edge
    lengths); "paper": the paper's form on its 240 inputs (Sec. 3, Sec. 4.2;
    the 24 geometry features of each curved cell from its vertices), params
    = (Ws, gammas, betas, means, stds), FP32 or BF16."""

    def __init__(self, box, ns, coords, params, dtype="bf16", device="cuda:0", shift=None, inv_scale=None,
                 indicator=False, fused=True, network="mlp"):
        self.box = L.Box.of(box)
        self.ns = L.NS.of(ns)
        self.dev = torch.device(device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.nf, self.nc, self.np = L.box_sizes(self.box)
        self.network = network
        if network == "paper":
            Ws = params[0]
            self.n_in, self.n_out = int(np.shape(Ws[0])[0]), int(np.shape(Ws[-1])[1])
            self.hidden = int(np.shape(Ws[0])[1])
            self.ldx = L.deepnet_widths(self.n_in, self.hidden, self.n_out)[0]
        else:
            self.n_in, self.n_out, self.ldx = L.LEVEL_IO[1]
            self.hidden = int(np.shape(params[0])[1])
        self.indicator = indicator
        # fused: the gather runs inside the network kernel
        self.fused = bool(fused) and network == "mlp"
        f32 = dict(dtype=torch.float32, device=self.dev)
        f64 = dict(dtype=torch.float64, device=self.dev)
        self.coords = torch.as_tensor(np.ascontiguousarray(coords, np.float64).ravel()).to(self.dev)
        # geometry inputs of the curved cells, fixed with the mesh
        self.geom = torch.zeros(3 * self.np, **f32)
        self.ws_q2 = torch.zeros(L.q2_workspace_bytes(self.box), dtype=torch.uint8, device=self.dev)
        L.dnnmg_q2_patch_features(self.box, self.coords, self.geom)
        if network == "paper":
            self.geo24 = torch.zeros(24 * self.np, **f32)
            L.dnnmg_q2_patch_features24(self.box, self.coords, self.geo24)
        self.xc = torch.zeros(4 * self.nc, **f64)
        self.xt = torch.zeros(4 * self.nf, **f32)
        self.vprev = torch.zeros(3 * self.nf, **f32)
        self.r = torch.zeros(4 * self.nf, **f32)
        self.xdtype = L.F32 if self.dtype == L.F32 else L.BF16
        self.X = torch.zeros(self.np * self.ldx, dtype=_TORCH[self.xdtype], device=self.dev)
        self.Y = torch.zeros(self.np * self.n_out, **f32)
        self.xcorr = torch.zeros(4 * self.nf, **f32)
        self.b = torch.zeros(4 * self.nf, **f32)
        self.bc = torch.zeros(4 * self.nc, **f64)
        if indicator:
            self.r2 = torch.zeros(4 * self.nf, **f32)
            self.norms = torch.zeros(2, **f64)
            self.ws_norm = torch.zeros(2 * L.norm2_workspace_bytes(), dtype=torch.uint8, device=self.dev)
        self.shift = None if shift is None else torch.as_tensor(np.asarray(shift, np.float32)).to(self.dev)
        self.inv_scale = None if inv_scale is None else torch.as_tensor(np.asarray(inv_scale, np.float32)).to(self.dev)
        if network == "paper":
            self.deep = L.DeepNet(self.dtype, *params, device=self.dev)
        else:
            W32 = [torch.as_tensor(np.asarray(params[2 * l], np.float32)).contiguous().to(self.dev) for l in range(3)]
            bias = [torch.as_tensor(np.asarray(params[2 * l + 1], np.float32)).contiguous().to(self.dev)
                    for l in range(3)]
            self.prepared = L.mlp_prepare(self.dtype, self.hidden, W32, bias, device=self.dev)
            self.net = self.prepared.net
        self.graph = None

    def load(self, xc, vprev):
        self.xc.copy_(torch.as_tensor(np.asarray(xc, np.float64).ravel()))
        self.vprev.copy_(torch.as_tensor(np.asarray(vprev, np.float32).ravel()))
        L.dnnmg_q2_rhs(self.box, self.ns, self.coords, self.vprev, self.b, ws=self.ws_q2)

    def step(self, stream=None):
        box, ns = self.box, self.ns
        L.dnnmg_q2_prolong(box, self.xc, self.xt, stream=stream)
        L.dnnmg_q2_residual_b(box, ns, self.coords, self.xt, self.b, self.r, ws=self.ws_q2, stream=stream)
        if self.network == "paper":
            L.dnnmg_patch_gather_paper_geom(box, self.geo24, self.xt, self.r, self.X, self.xdtype, self.ldx,
                                            self.shift, self.inv_scale, stream=stream)
            L.dnnmg_deepnet_forward(self.deep, self.np, self.X, self.ldx, self.Y, stream=stream)
        elif self.fused:
            L.dnnmg_patch_gather_forward_geom(box, self.net, self.geom, self.xt, self.r, self.Y, self.shift,
                                              self.inv_scale, stream=stream)
        else:
            L.dnnmg_patch_gather_geom(box, self.geom, self.xt, self.r, self.X, self.xdtype, self.ldx, self.shift,
                                      self.inv_scale, stream=stream)
            L.dnnmg_patch_forward(self.net, self.np, self.X, self.ldx, self.Y, stream=stream)
        L.dnnmg_scatter_avg(box, self.Y, self.xcorr, vbase=self.xt, stream=stream)
        if self.indicator:
            # the indicator's residual and the next right-hand side at x_corr in one pass
            L.dnnmg_q2_residual_rhs(box, ns, self.coords, self.xcorr, self.b, self.r2, self.b, ws=self.ws_q2,
                                    stream=stream)
            L.dnnmg_norm2_pair_f64(self.r, self.r2, self.norms, self.ws_norm, stream=stream)
        else:
            L.dnnmg_q2_rhs(box, ns, self.coords, self.xcorr, self.b, ws=self.ws_q2, stream=stream)
        L.dnnmg_q2_restrict(box, self.b, self.bc, stream=stream)

    def capture(self):
        self.graph = L.capture_graph(self.step, device=self.dev)
        return self.graph

    def replay(self, stream=None):
        self.graph.replay(stream)

    def run_numpy(self, xc, vprev):
        self.load(xc, vprev)
        b_in = self.b.cpu().numpy().reshape(4, -1).astype(np.float64)
        self.step()
        torch.cuda.synchronize(self.dev)
        xt = self.xt.cpu().numpy().reshape(4, -1).astype(np.float64)
        xcorr = self.xcorr.cpu().numpy().reshape(4, -1).astype(np.float64)
        out = {
            "b_in": b_in,
            "xt": xt,
            "r": self.r.cpu().numpy().reshape(4, -1).astype(np.float64),
            "Y": self.Y.cpu().numpy().reshape(-1, self.n_out).astype(np.float64),
            "vcorr": xcorr[:3],
            "d": xcorr[:3] - xt[:3],
            "b": self.b.cpu().numpy().reshape(4, -1).astype(np.float64),
            "bc": self.bc.cpu().numpy().reshape(4, -1),
        }
        if self.indicator:
            n = self.norms.cpu().numpy()
            out["r2"] = self.r2.cpu().numpy().reshape(4, -1).astype(np.float64)
            out["eta"] = float(np.sqrt(n[1] / n[0])) if n[0] > 0 else float("inf")
        return out
