"""Benchmark of the DNN-MG fine-level correction step on one MI355X.

One step = prolongation -> fine residual -> patch gather -> patch network ->
multiplicity-averaged extension -> right-hand side -> restriction (the hot
path after the coarse solve), captured in one HIP graph and replayed.

Default workload: the single-simulation channel, coarse 64x16x16 cells
(16,384 patches), fine 128x32x32 cells (140,481 nodes), FP32 stencils and a
BF16 network 165-256-256-81.  Prints one JSON line; `value` is patches/s.
Also reported: the same step with an FP32 network, and the large channel
(131,072 patches, FP8 network of width 512) with the residual indicator.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3  # published vector FP32 (packed FMA); non-packed issue is half
BF16_MFMA_PEAK_TFLOPS = 2500.0
PMC_COPY_MIB = 256  # plain copy of known size that calibrates the HBM byte counters


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-variants", action="store_true", help="only the default workload")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="run only the dominant kernel and a plain copy a few times (for rocprofv3 --pmc)")
    ap.add_argument("--scale-only", action="store_true",
                    help="run only the per-kernel measurements on the large channel (for rocprofv3)")
    return ap.parse_args()


RESIDUAL_SOURCES = ("residual.hip", "common.hpp", "common.hip")


def src_hash(*names):
    h = hashlib.sha256()
    for n in names:
        h.update(open(os.path.join(ROOT, "paper_2307_14837_amd", "csrc", n), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(entry, workload):
    """HBM bytes per launch of an entry point from the committed rocprofv3 PMC
    summary, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"pmc_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    k = rec.get("entries", {}).get(entry)
    if not k or k.get("src_hash") != src_hash(*RESIDUAL_SOURCES):
        return None
    return k.get("bytes_per_launch")


def pmc_probe():
    """The dominant entry point (prolongation + residual of the default
    workload, in the form against the carried right-hand side, and in the
    form that reads v_prev), then a plain device copy of PMC_COPY_MIB MiB,
    three launches each, for counter runs."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L

    w = syn.cfg2()
    st, _, _ = build_step(w, "bf16")
    for _ in range(3):
        L.dnnmg_prolong_residual(st.box, st.ns, st.xc, st.vprev, st.xt, st.r)
    for _ in range(3):
        L.dnnmg_prolong_residual_b(st.box, st.ns, st.xc, st.b, st.xt, st.r)
    torch.cuda.synchronize()
    n = PMC_COPY_MIB * 2**20 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": w.name, "copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n,
                      "src_hash": src_hash(*RESIDUAL_SOURCES)}), flush=True)


def time_graph(st, steps, warmup):
    import torch

    st.capture()
    for _ in range(warmup):
        st.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(steps):
        st.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


def time_kernel(fn, reps):
    """Average duration of one launch of fn(): `reps` back-to-back launches are
    captured in one HIP graph (no host launch gaps) and timed with HIP events
    on the stream the graph is replayed on."""
    import torch

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def build_step(w, dtype, seed=0, indicator=False, theta=1.0):
    import dnnmg_synth as syn
    from paper_2307_14837_amd import stepper

    inp = syn.step_inputs(w, seed=seed)
    params = syn.mlp_params(165, w.hidden, 81, seed=seed)
    st = stepper.CorrectionStep(w.box, w.ns, params, dtype=dtype, indicator=indicator, theta=theta)
    st.load(inp.xc, inp.vprev)
    return st, inp, params


def run_variant(w, dtype, steps, warmup, indicator=False, fallback="never"):
    """indicator: the residual test runs every step; fallback "never"
    (threshold infinite: test only) or "always" (threshold 0: the
    fallback sweeps replace the correction every step)."""
    theta = float("inf") if fallback == "never" else 0.0
    st, inp, params = build_step(w, dtype, indicator=indicator, theta=theta)
    ms, wall = time_graph(st, steps, warmup)
    return {"workload": w.name, "dtype": dtype, "indicator": indicator,
            "fallback": fallback if indicator else None, "ms_per_step": ms,
            "patches_per_s": st.np / (ms * 1e-3), "fine_dof_per_s": 4 * st.nf / (ms * 1e-3)}


def run_batched(dtype, steps, warmup):
    """The 32 uneven periodic boxes in one plan: fused persistent network
    stage, autotuned, whole step in one HIP graph."""
    import dnnmg_synth as syn
    from paper_2307_14837_amd import batched

    boxes = syn.cfg3_boxes(seed=0)
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=0)
    xcs, vps = [], []
    for i, b in enumerate(boxes):
        inp = syn.step_inputs(syn.Workload("b", b, ns, 256, dtype, "fourier"), seed=i)
        xcs.append(inp.xc)
        vps.append(inp.vprev)
    bs = batched.BatchedStep(boxes, ns, params, dtype=dtype)
    bs.load(xcs, vps)
    ppt, grid = bs.autotune(reps=5)
    ms, _ = time_graph(bs, steps, warmup)
    npch, nf = bs.plan.n_patches, bs.plan.n_fine
    return {"workload": "cfg3_32_periodic_boxes", "boxes": len(boxes), "patches": npch, "fine_nodes": nf,
            "dtype": dtype, "fused_batched": True, "autotuned": {"patches_per_tile": ppt, "grid": grid},
            "ms_per_step": ms, "patches_per_s": npch / (ms * 1e-3), "fine_dof_per_s": 4 * nf / (ms * 1e-3)}


def run_per_box_plain(dtype, steps, warmup):
    """The same 32 boxes as separate plain steps (unfused gather, FP32 network),
    all 32 captured in one HIP graph."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import stepper

    boxes = syn.cfg3_boxes(seed=0)
    ns = syn.NSParams(1e-3, 0.01)
    params = syn.mlp_params(165, 256, 81, seed=0)
    sts = []
    for i, b in enumerate(boxes):
        inp = syn.step_inputs(syn.Workload("b", b, ns, 256, dtype, "fourier"), seed=i)
        st = stepper.CorrectionStep(b, ns, params, dtype=dtype, fused=False)
        st.load(inp.xc, inp.vprev)
        sts.append(st)

    class All:
        def step(self):
            for st in sts:
                st.step()

        def capture(self):
            self.g = L.capture_graph(self.step)

        def replay(self):
            self.g.replay()

    ms, _ = time_graph(All(), steps, warmup)
    npch = sum(b.n_patches for b in boxes)
    nf = sum(b.n_fine for b in boxes)
    return {"workload": "cfg3_32_periodic_boxes", "boxes": len(boxes), "patches": npch, "dtype": dtype,
            "fused_batched": False, "ms_per_step": ms, "patches_per_s": npch / (ms * 1e-3),
            "fine_dof_per_s": 4 * nf / (ms * 1e-3)}


def run_training(steps):
    """One AdamW step of the patch network at the training batch size
    (65,536 patches, width 256, BF16 compute, FP32 master weights)."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import train

    n, H = 65536, 256
    params = syn.mlp_params(165, H, 81, seed=0)
    tr = train.PatchTrainer(params, dtype="bf16", max_batch=n)
    rng = np.random.default_rng(0)
    X = torch.zeros(n * 192, dtype=torch.bfloat16, device="cuda")
    Xv = torch.as_tensor(rng.standard_normal((n, 165)).astype(np.float32))
    X.view(n, 192)[:, :165] = Xv.to("cuda").to(torch.bfloat16)
    T = torch.as_tensor(rng.standard_normal((n, 81)).astype(np.float32)).view(-1).to("cuda")
    for _ in range(3):
        tr.step(X, T, n)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        tr.step(X, T, n)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    from paper_2307_14837_amd import flops

    fl = 3 * flops.mlp_flops_per_patch(H) * n  # forward + backward (about 2x forward)
    return {"workload": "training_batch_65536_width256",
            "dtype": "bf16 forward and backward products, fp32 accumulation and master weights",
            "ms_per_step": ms, "patches_per_s": n / (ms * 1e-3), "approx_tflops": fl / (ms * 1e-3) / 1e12}


def kernels_at_scale():
    """The hot-path kernels on the large channel (coarse 128x32x32: 131,072
    patches, 1,085,825 fine nodes), each timed alone (50 graph-captured
    launches): HBM-bound stencils as achieved GB/s of their algorithmic bytes,
    VALU kernels as TFLOP/s, network forwards as TFLOP/s."""
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import flops

    w = syn.cfg5()
    st, inp, params = build_step(w, "bf16")
    st.step()
    torch.cuda.synchronize()
    nf, npch = st.nf, st.np
    ncell = 8 * npch
    reps = 50
    out = {"workload": w.name, "fine_nodes": nf, "patches": npch}
    B = flops.BYTES_PER_FINE_NODE

    def hbm(name, fn, nbytes):
        # the kernel's algorithmic bytes per second, beside a plain device
        # copy moving the same number of bytes (the practical ceiling at
        # this size: launch and ramp included)
        t = time_kernel(fn, reps)
        a = torch.empty(int(nbytes) // 8, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        tc = time_kernel(lambda: b.copy_(a), reps)
        out[name] = {"ms": t, "GB/s": nbytes / (t * 1e-3) / 1e9, "copy_same_bytes_GB/s": 8 * a.numel() / (tc * 1e-3) / 1e9}

    hbm("prolong", lambda: L.dnnmg_prolong(st.box, st.xc, st.xt), B["prolong"] * nf)
    for form, tag in ((L.SCATTER_NODES, "scatter_nodes"), (L.SCATTER_TILED, "scatter_tiled")):
        hbm(tag, lambda: L.dnnmg_scatter_avg_form(st.box, st.Y, st.xcorr, form, vbase=st.xt), B["scatter"] * nf)
    hbm("restrict", lambda: L.dnnmg_restrict(st.box, st.b, st.bc), B["restrict"] * nf)
    hbm("gather_bf16", lambda: L.dnnmg_patch_gather(st.box, st.xt, st.r, st.X, st.xdtype, 192, st.shift,
                                                    st.inv_scale), flops.gather_bytes_per_patch(2) * npch)
    t = time_kernel(lambda: L.dnnmg_prolong_residual(st.box, st.ns, st.xc, st.vprev, st.xt, st.r), reps)
    out["prolong_residual"] = {"ms": t, "TFLOP/s": flops.prolong_residual_flops_per_cell() * ncell / (t * 1e-3) / 1e12}
    t = time_kernel(lambda: L.dnnmg_prolong_residual_b(st.box, st.ns, st.xc, st.b, st.xt, st.r), reps)
    out["prolong_residual_b"] = {"ms": t,
                                 "TFLOP/s": flops.prolong_residual_b_flops_per_cell() * ncell / (t * 1e-3) / 1e12}
    t = time_kernel(lambda: L.dnnmg_rhs(st.box, st.ns, st.xcorr, st.b), reps)
    out["rhs"] = {"ms": t, "TFLOP/s": flops.rhs_flops_per_cell() * ncell / (t * 1e-3) / 1e12}
    fl = flops.mlp_flops_per_patch(w.hidden) * npch
    for dtype in ("bf16", "fp8"):
        s2, _, _ = build_step(w, dtype)
        L.dnnmg_patch_gather(s2.box, s2.xt, s2.r, s2.X, s2.xdtype, 192, s2.shift, s2.inv_scale)
        for tp in (32, 64):
            t = time_kernel(lambda: L.dnnmg_patch_forward_tiles(s2.net, npch, s2.X, 192, s2.Y, tp), reps)
            out[f"forward_{dtype}_{tp}"] = {"ms": t, "TFLOP/s": fl / (t * 1e-3) / 1e12}
    return out


def accuracy(w, dtype):
    """rel-L2 of the corrected velocity correction d and of b^L against the
    FP64 oracle on the same inputs (test infrastructure)."""
    import oracle

    st, inp, params = build_step(w, dtype)
    out = st.run_numpy(inp.xc, inp.vprev)
    p32 = [np.asarray(p, np.float32).astype(np.float64) for p in params]
    ref = oracle.correction_step(w.box, w.ns, p32, inp.xc, out["vprev32"])
    rel = lambda a, b: float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    return {"d": rel(out["d"], ref["d"]), "r": rel(out["r"], ref["r"]), "bc": rel(out["bc"], ref["bc"])}


def cpu_baseline(w):
    """The oracle as it stands, one full correction step of the same workload
    on one host core (the oracle is single-threaded C)."""
    import dnnmg_synth as syn
    import oracle

    inp = syn.step_inputs(w, seed=0)
    params = [np.asarray(p, np.float32).astype(np.float64) for p in syn.mlp_params(165, w.hidden, 81, seed=0)]
    oracle.lib()
    t0 = time.perf_counter()
    oracle.correction_step(w.box, w.ns, params, inp.xc, inp.vprev)
    dt = time.perf_counter() - t0
    return {"value": w.box.n_patches / dt, "unit": "patches/s", "cores": 1, "kind": "oracle",
            "sample": f"one full correction step of {w.name} ({w.box.n_patches} patches) in FP64, "
                      f"{dt:.2f} s"}


def main():
    args = parse()
    if args.pmc_probe:
        pmc_probe()
        return
    if args.scale_only:
        print(json.dumps({"kernels_at_scale": kernels_at_scale()}), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import dnnmg_synth as syn
    from paper_2307_14837_amd import _lib as L
    from paper_2307_14837_amd import flops

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    w = syn.cfg2()
    st, inp, params = build_step(w, "bf16")
    print(f"[bench] {w.name}: {st.np} patches, {st.nf} fine nodes; timing {args.steps} graph replays",
          file=sys.stderr, flush=True)
    ms, wall = time_graph(st, args.steps, args.warmup)

    # dominant kernel: prolongation + fine residual against the carried
    # right-hand side (VALU bound), timed live with HIP events on the stream
    # it runs on
    reps = 50
    res_ms = time_kernel(lambda: L.dnnmg_prolong_residual_b(st.box, st.ns, st.xc, st.b, st.xt, st.r), reps)
    ncells = 8 * st.np
    flop = flops.prolong_residual_b_flops_per_cell() * ncells
    achieved = flop / (res_ms * 1e-3) / 1e12
    traffic = traffic_from_profile("dnnmg_prolong_residual_b", w.name)
    L.dnnmg_patch_gather(st.box, st.xt, st.r, st.X, st.xdtype, 192, st.shift, st.inv_scale)
    kernel_ms = {
        "prolong_residual_b": res_ms,
        "prolong_residual": time_kernel(lambda: L.dnnmg_prolong_residual(st.box, st.ns, st.xc, st.vprev, st.xt,
                                                                         st.r), reps),
        "residual": time_kernel(lambda: L.dnnmg_residual(st.box, st.ns, st.xt, st.vprev, st.r, st.ws_res), reps),
        "prolong": time_kernel(lambda: L.dnnmg_prolong(st.box, st.xc, st.xt), reps),
        "gather_forward_fused": time_kernel(lambda: L.dnnmg_patch_gather_forward(st.box, st.net, st.xt, st.r, st.Y,
                                                                                st.shift, st.inv_scale), reps),
        "gather": time_kernel(lambda: L.dnnmg_patch_gather(st.box, st.xt, st.r, st.X, st.xdtype, 192,
                                                          st.shift, st.inv_scale), reps),
        "forward": time_kernel(lambda: L.dnnmg_patch_forward(st.net, st.np, st.X, 192, st.Y), reps),
        "scatter": time_kernel(lambda: L.dnnmg_scatter_avg(st.box, st.Y, st.xcorr, vbase=st.xt), reps),
        "rhs": time_kernel(lambda: L.dnnmg_rhs(st.box, st.ns, st.xcorr, st.b), reps),
        "restrict": time_kernel(lambda: L.dnnmg_restrict(st.box, st.b, st.bc), reps),
    }
    fwd_tiles = {}
    for tp in (16, 32, 64):
        fwd_tiles[tp] = time_kernel(lambda: L.dnnmg_patch_forward_tiles(st.net, st.np, st.X, 192, st.Y, tp), reps)
    kernel_ms["forward_by_tile"] = fwd_tiles
    mlp_flop = flops.mlp_flops_per_patch(256) * st.np
    out = {
        "metric": "DNN-MG correction step throughput (patches/s; fine DOF/s also given)",
        "value": st.np / (ms * 1e-3),
        "unit": "patches/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": w.name, "patches": st.np, "fine_nodes": st.nf, "fine_dofs": 4 * st.nf,
                   "network": "165-256-256-81 tanh, BF16 MFMA, FP32 accumulate",
                   "stencils": "FP32 (prolongation from FP64, restriction to FP64)",
                   "parallelism": "1 GPU", "graph": "hipGraph replay of the whole step"},
        "fine_dof_per_s": 4 * st.nf / (ms * 1e-3),
        "roofline": {"kernel": "dnnmg_prolong_residual_b", "bound": "alu", "achieved": achieved,
                     "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic,
                     "avg_launch_ms": res_ms, "flop_per_launch": flop},
        "kernel_ms": kernel_ms,
        "mlp_tflops": mlp_flop / (kernel_ms["forward"] * 1e-3) / 1e12,
        "wall_s_timed": wall,
    }
    if not args.no_variants:
        print("[bench] variants: fp32 network, indicator, large FP8 channel", file=sys.stderr, flush=True)
        out["variants"] = [
            run_variant(w, "fp32", args.steps, args.warmup),
            run_variant(w, "bf16", args.steps, args.warmup, indicator=True, fallback="never"),
            run_variant(w, "bf16", args.steps, args.warmup, indicator=True, fallback="always"),
            run_variant(syn.cfg5(), "fp8", max(args.steps // 4, 10), max(args.warmup // 4, 3), indicator=True),
            run_variant(syn.cfg5(), "bf16", max(args.steps // 4, 10), max(args.warmup // 4, 3)),
            run_batched("bf16", max(args.steps // 4, 10), max(args.warmup // 4, 3)),
            run_per_box_plain("fp32", max(args.steps // 4, 10), max(args.warmup // 4, 3)),
            run_training(20),
        ]
        print("[bench] kernels on the large channel", file=sys.stderr, flush=True)
        out["kernels_at_scale"] = kernels_at_scale()
        print("[bench] accuracy vs oracle", file=sys.stderr, flush=True)
        out["accuracy_rel_l2"] = {"bf16": accuracy(w, "bf16"), "fp32": accuracy(w, "fp32")}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
