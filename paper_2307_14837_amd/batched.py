"""Batched correction step over many independent boxes of uneven size (one
plan, five launches per step whatever the number of boxes), with the
autotuned network stage and HIP-graph capture.  By default the step carries
the right-hand side: each step's residual is r = b - A(x~) with the b the
previous step computed (load() computes the first one from vprev)."""
from __future__ import annotations

import numpy as np
import torch

from . import _lib as L
from .stepper import DTYPES


class BatchedStep:
    def __init__(self, boxes, ns, params, dtype="bf16", device="cuda:0", shift=None, inv_scale=None,
                 carry_rhs=True):
        self.dev = torch.device(device)
        self.carry_rhs = bool(carry_rhs)
        self.boxes = [L.Box.of(b) for b in boxes]
        self.sizes = [L.box_sizes(b) for b in self.boxes]
        self.plan = L.Plan(self.boxes, ns, device=device)
        self.dtype = DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        nf, nc, npch = self.plan.n_fine, self.plan.n_coarse, self.plan.n_patches
        f32 = dict(dtype=torch.float32, device=self.dev)
        self.bufs = {
            "xc": torch.zeros(4 * nc, dtype=torch.float64, device=self.dev),
            "vprev": torch.zeros(3 * nf, **f32), "xt": torch.zeros(4 * nf, **f32),
            "r": torch.zeros(4 * nf, **f32), "Y": torch.zeros(npch * L.N_OUT, **f32),
            "xcorr": torch.zeros(4 * nf, **f32), "b": torch.zeros(4 * nf, **f32),
            "bc": torch.zeros(4 * nc, dtype=torch.float64, device=self.dev),
        }
        self.shift = None if shift is None else torch.as_tensor(np.asarray(shift, np.float32)).to(self.dev)
        self.inv_scale = None if inv_scale is None else torch.as_tensor(np.asarray(inv_scale, np.float32)).to(self.dev)
        H = int(np.shape(params[0])[1])
        W32 = [torch.as_tensor(np.asarray(params[2 * l], np.float32)).contiguous().to(self.dev) for l in range(3)]
        bias = [torch.as_tensor(np.asarray(params[2 * l + 1], np.float32)).contiguous().to(self.dev) for l in range(3)]
        self.prepared = L.mlp_prepare(self.dtype, H, W32, bias, device=self.dev)
        self.net = self.prepared.net
        self.graph = None

    # per-box views of the batch layout
    def _offsets(self):
        of = oc = op = 0
        for nf, nc, npch in self.sizes:
            yield of, oc, op, nf, nc, npch
            of += nf
            oc += nc
            op += npch

    def load(self, xcs, vprevs):
        xc = np.concatenate([np.asarray(x, np.float64).reshape(4, -1).ravel() for x in xcs])
        vp = np.concatenate([np.asarray(v, np.float32).reshape(3, -1).ravel() for v in vprevs])
        self.bufs["xc"].copy_(torch.as_tensor(xc))
        self.bufs["vprev"].copy_(torch.as_tensor(vp))
        if self.carry_rhs:
            # the previous velocity in the 4-component layout (xcorr is
            # scratch until the step writes it), then its right-hand side
            v4 = self.bufs["xcorr"]
            for of, oc, op, nf, nc, npch in self._offsets():
                v4[4 * of:4 * of + 3 * nf].copy_(self.bufs["vprev"][3 * of:3 * of + 3 * nf])
            self.plan.rhs(v4, self.bufs["b"])

    def step(self, stream=None):
        if self.carry_rhs:
            self.plan.step_b(self.net, self.bufs, self.shift, self.inv_scale, stream=stream)
        else:
            self.plan.step(self.net, self.bufs, self.shift, self.inv_scale, stream=stream)

    def autotune(self, reps=5):
        self.plan.autotune(self.net, self.bufs, self.shift, self.inv_scale, reps=reps)
        return self.plan.choice()

    def capture(self):
        self.graph = L.capture_graph(self.step, device=self.dev)
        return self.graph

    def replay(self, stream=None):
        self.graph.replay(stream)

    def results(self):
        """Per-box numpy outputs: xt, xcorr, bc, Y."""
        torch.cuda.synchronize(self.dev)
        b = {k: v.cpu().numpy() for k, v in self.bufs.items()}
        out = []
        for of, oc, op, nf, nc, npch in self._offsets():
            out.append({"xt": b["xt"][4 * of:4 * (of + nf)].reshape(4, nf),
                        "xcorr": b["xcorr"][4 * of:4 * (of + nf)].reshape(4, nf),
                        "bc": b["bc"][4 * oc:4 * (oc + nc)].reshape(4, nc),
                        "Y": b["Y"][81 * op:81 * (op + npch)].reshape(npch, 81)})
        return out
